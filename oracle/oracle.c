/*
 * oracle.c -- CPU reference for the direct ghost-cell method.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product library.  Shares no
 * code with the GPU path.  Plain C99 in FP64, built with -ffp-contract=off.
 *
 * The method (paper sections cited per function):
 *   Sec. 3.1  classify cells by centre (fluid 0 / solid 1), tag ghost cells
 *             (CGC +2; HGC +2 / -2 via the signed distance psi, the normal
 *             cell thickness Delta n, and the reclassification rule).
 *   Sec. 3.2  ghost-to-ghost dependency graph, Kahn levels L1..Ln.
 *   Sec. 4/5  Dirichlet and Neumann reconstruction relations (2D, 3D) and
 *             their Vandermonde derivation (Appendix A).
 *   Sec. 6    boundary value and Cartesian gradient at S, forces.
 *   Sec. 7    extended-stencil multipliers r_i (CGC_ES).
 * Where the paper is silent the readings are: face neighbours for
 * "adjacent"; reclassification judged on the centre classification; S is the
 * closest boundary point with the analytic normal there; sgn(0) = +1; zero
 * normal components remove (and do not read) the displaced stencil points;
 * within a level ghosts are ordered by linear index.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXD 3

struct orc_plan {
  orc_grid g;
  orc_shape s;
  double* coef;
  int scheme, dim;
  int64_t ncell, nif, ng;
  int32_t nlev;
  int8_t* tag;
  int32_t* lev_off;     /* [nlev+1] */
  /* canonical order (level, linear index) */
  int64_t* cell;
  int32_t* level;
  double* delta;        /* [dim][ng] : x_s - x_c */
  double* nrm;          /* [dim][ng] : unit normal into the fluid at S */
  double* psi;          /* [ng] */
  int32_t* r;           /* [dim][ng] : stencil multipliers */
  int32_t* e;           /* [dim][ng] : sgn(n_i), sgn(0) = +1 */
  int64_t* sten;        /* [ng][7] : stencil cells, -1 = skipped */
  /* linear-index order lookup */
  int64_t* sorted_cell; /* [ng] */
  int64_t* sorted_pos;  /* [ng] canonical position */
  /* coupled units (strongly connected components of more than one ghost) */
  int32_t nblk, maxblk;
  int32_t* blk;         /* [ng] unit id or -1 */
  int32_t* blk_off;     /* [nblk+1] */
  int64_t* blk_mem;     /* members, canonical positions, ascending */
  double margins[7];
  double* faces[3];     /* owned copies of a stretched grid's faces */
};


/* ------------------------------------------------------------------------- */
/* grid helpers                                                              */
/* ------------------------------------------------------------------------- */

static double centre(const orc_grid* g, int ax, int64_t i) {
  if (g->faces[ax]) return 0.5 * (g->faces[ax][i] + g->faces[ax][i + 1]);
  return g->lo[ax] + ((double)i + 0.5) * g->h[ax];
}

/* local spacing of cell i along axis ax: its width */
static double width(const orc_grid* g, int ax, int64_t i) {
  if (g->faces[ax]) return g->faces[ax][i + 1] - g->faces[ax][i];
  return g->h[ax];
}

/* x_2 - x_1 along axis ax for a stencil from cell i displaced by er cells
 * (stretched: the difference of the two centres; a displacement off the grid,
 * possible only along an axis the normal does not leave, uses the width) */
static double span(const orc_grid* g, int ax, int64_t i, int er) {
  if (!g->faces[ax]) return (double)er * g->h[ax];
  if (i + er < 0 || i + er >= g->n[ax]) return (double)er * width(g, ax, i);
  return centre(g, ax, i + er) - centre(g, ax, i);
}

/* index of the cell holding coordinate x along axis ax (outside the grid:
 * below 0 or at least n) */
static int64_t cell_of(const orc_grid* g, int ax, double x) {
  if (!g->faces[ax]) return (int64_t)floor((x - g->lo[ax]) / g->h[ax]);
  const double* f = g->faces[ax];
  const int64_t n = g->n[ax];
  if (x < f[0]) return -1;
  if (x >= f[n]) return n;
  int64_t lo = 0, hi = n - 1;   /* the last i with f[i] <= x */
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) / 2;
    if (f[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

static void unlinear(const orc_grid* g, int64_t c, int64_t ijk[3]) {
  ijk[0] = c % g->n[0];
  ijk[1] = (c / g->n[0]) % g->n[1];
  ijk[2] = (g->dim == 3) ? c / (g->n[0] * g->n[1]) : 0;
}

static int64_t linear(const orc_grid* g, const int64_t ijk[3]) {
  return ijk[0] + g->n[0] * (ijk[1] + g->n[1] * (g->dim == 3 ? ijk[2] : 0));
}

/* Stencil points in the paper's order: 2D P1=(x2,y1) P2=(x1,y2) P3=(x2,y2);
 * 3D P1..P7 = {x},{y},{z},{x,y},{y,z},{x,z},{x,y,z} (Sec. 4, Sec. 5). */
static const int SUB2[3][3] = {{1, 0, 0}, {0, 1, 0}, {1, 1, 0}};
static const int SUB3[7][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0},
                               {0, 1, 1}, {1, 0, 1}, {1, 1, 1}};

static const int* subset(int dim, int k) { return dim == 2 ? SUB2[k] : SUB3[k]; }
static int npts(int dim) { return dim == 2 ? 3 : 7; }

/* ------------------------------------------------------------------------- */
/* forward-mode dual numbers (value + gradient in R^3), used to evaluate the */
/* spherical-harmonic radius and its gradient without trigonometry          */
/* ------------------------------------------------------------------------- */

typedef struct { double v, d[3]; } dual;

static dual dc(double a) { dual r = {a, {0, 0, 0}}; return r; }
static dual dadd(dual a, dual b) {
  dual r; r.v = a.v + b.v;
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
static dual dsub(dual a, dual b) {
  dual r; r.v = a.v - b.v;
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
static dual dmul(dual a, dual b) {
  dual r; r.v = a.v * b.v;
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
static dual dscale(dual a, double s) {
  dual r; r.v = a.v * s;
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] * s;
  return r;
}
static dual ddiv(dual a, dual b) {
  dual r; r.v = a.v / b.v;
  for (int i = 0; i < 3; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
static dual dsqrt(dual a) {
  dual r; r.v = sqrt(a.v);
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] / (2.0 * r.v);
  return r;
}

static double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= (double)i;
  return f;
}

/* Real Schmidt semi-normalised harmonic Y_lm at direction v/|v| (no
 * Condon-Shortley phase):
 *   Y_lm = N_lm P_l^|m|(cos theta) {cos m phi (m>=0), sin |m| phi (m<0)},
 *   N_l0 = 1, N_lm = sqrt(2 (l-m)!/(l+m)!).
 * Written as N_lm * (d^m P_l/dt^m)(z/rho) * {Re,Im}(((x + i y)/rho)^|m|), which
 * is the same function with sin^m(theta) e^{i m phi} = ((x+iy)/rho)^m.        */
static dual sh_dual(int l, int m, const dual v[3]) {
  int am = m < 0 ? -m : m;
  dual rho = dsqrt(dadd(dadd(dmul(v[0], v[0]), dmul(v[1], v[1])), dmul(v[2], v[2])));
  dual t = ddiv(v[2], rho);
  dual ux = ddiv(v[0], rho), uy = ddiv(v[1], rho);
  /* d^m P_l / dt^m by the Legendre recurrence in l at fixed m */
  double dfact = 1.0;
  for (int i = 1; i <= 2 * am - 1; i += 2) dfact *= (double)i;
  dual pmm = dc(dfact), p;
  if (l == am) {
    p = pmm;
  } else {
    dual pm1 = dscale(dmul(t, pmm), (double)(2 * am + 1));
    if (l == am + 1) {
      p = pm1;
    } else {
      dual a = pmm, b = pm1;
      for (int ll = am + 2; ll <= l; ++ll) {
        dual c = dscale(dsub(dscale(dmul(t, b), (double)(2 * ll - 1)),
                             dscale(a, (double)(ll + am - 1))),
                        1.0 / (double)(ll - am));
        a = b; b = c;
      }
      p = b;
    }
  }
  /* ((x + i y)/rho)^|m| */
  dual re = dc(1.0), im = dc(0.0);
  for (int i = 0; i < am; ++i) {
    dual nre = dsub(dmul(re, ux), dmul(im, uy));
    dual nim = dadd(dmul(re, uy), dmul(im, ux));
    re = nre; im = nim;
  }
  double N = (am == 0) ? 1.0 : sqrt(2.0 * factorial(l - am) / factorial(l + am));
  return dscale(dmul(p, m >= 0 ? re : im), N);
}

double orc_sh_basis(int l, int m, const double* v) {
  dual dv[3];
  for (int i = 0; i < 3; ++i) { dv[i] = dc(v[i]); dv[i].d[i] = 1.0; }
  return sh_dual(l, m, dv).v;
}

/* r(omega) and its gradient with respect to the (unnormalised) direction v. */
static dual shstar_radius(const orc_shape* s, const double v[3]) {
  dual dv[3];
  for (int i = 0; i < 3; ++i) { dv[i] = dc(v[i]); dv[i].d[i] = 1.0; }
  int L = (int)floor(sqrt((double)s->ncoef) + 1e-9) - 1;
  dual sum = dc(1.0);
  for (int l = 0; l <= L; ++l)
    for (int m = -l; m <= l; ++m) {
      double a = s->coef[l * l + l + m];
      if (a != 0.0) sum = dadd(sum, dscale(sh_dual(l, m, dv), a));
    }
  return dscale(sum, s->r0);
}

/* r(omega) alone: the same recurrences in plain doubles (the value parts of
 * the dual-number operations above are these very operations). */
static double sh_value(int l, int m, const double v[3]) {
  int am = m < 0 ? -m : m;
  double rho = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  double t = v[2] / rho, ux = v[0] / rho, uy = v[1] / rho;
  double dfact = 1.0;
  for (int i = 1; i <= 2 * am - 1; i += 2) dfact *= (double)i;
  double p;
  if (l == am) {
    p = dfact;
  } else {
    double pm1 = (t * dfact) * (double)(2 * am + 1);
    if (l == am + 1) {
      p = pm1;
    } else {
      double a = dfact, b = pm1;
      for (int ll = am + 2; ll <= l; ++ll) {
        double c = ((t * b) * (double)(2 * ll - 1) - a * (double)(ll + am - 1)) *
                   (1.0 / (double)(ll - am));
        a = b; b = c;
      }
      p = b;
    }
  }
  double re = 1.0, im = 0.0;
  for (int i = 0; i < am; ++i) {
    double nre = re * ux - im * uy;
    double nim = re * uy + im * ux;
    re = nre; im = nim;
  }
  double N = (am == 0) ? 1.0 : sqrt(2.0 * factorial(l - am) / factorial(l + am));
  return (p * (m >= 0 ? re : im)) * N;
}

static double shstar_radius_value(const orc_shape* s, const double v[3]) {
  int L = (int)floor(sqrt((double)s->ncoef) + 1e-9) - 1;
  double sum = 1.0;
  for (int l = 0; l <= L; ++l)
    for (int m = -l; m <= l; ++m) {
      double a = s->coef[l * l + l + m];
      if (a != 0.0) sum = sum + sh_value(l, m, v) * a;
    }
  return sum * s->r0;
}

/* 2D star: r(theta), r'(theta), r''(theta). */
static void star_radius(const orc_shape* s, double th, double* r, double* r1,
                        double* r2) {
  double a = 1.0, b = 0.0, c = 0.0;
  for (int k = 0; k < s->ncoef; ++k) {
    double A = s->coef[2 * k], B = s->coef[2 * k + 1];
    double ck = cos(k * th), sk = sin(k * th);
    a += A * ck + B * sk;
    b += (double)k * (-A * sk + B * ck);
    c += -(double)(k * k) * (A * ck + B * sk);
  }
  *r = s->r0 * a; *r1 = s->r0 * b; *r2 = s->r0 * c;
}

/* ------------------------------------------------------------------------- */
/* airfoil: symmetric four-digit thickness, closed trailing edge            */
/* ------------------------------------------------------------------------- */

/* half thickness y_t(x) for 0 <= x <= 1 (unit chord) */
static double naca_yt(double t, double x) {
  double sx = sqrt(x);
  return 5.0 * t * (0.2969 * sx - 0.1260 * x - 0.3516 * x * x +
                    0.2843 * x * x * x - 0.1036 * x * x * x * x);
}

/* Contour parameter s in [-1, 1]: x = s^2 (chord units), y = sgn(s) y_t(s^2).
 * Returns the point and first/second derivatives in the body frame.        */
static void naca_curve(double t, double s, double X[2], double D1[2],
                       double D2[2]) {
  double as = fabs(s), sg = s < 0 ? -1.0 : 1.0;
  double s2 = s * s;
  X[0] = s2;
  /* y = 5t (0.2969 s - sg (0.1260 s^2 + 0.3516 s^4 - 0.2843 s^6 + 0.1036 s^8)) */
  double poly = 0.1260 * s2 + 0.3516 * s2 * s2 - 0.2843 * s2 * s2 * s2 +
                0.1036 * s2 * s2 * s2 * s2;
  double dpoly = 2 * 0.1260 * s + 4 * 0.3516 * s2 * s - 6 * 0.2843 * s2 * s2 * s +
                 8 * 0.1036 * s2 * s2 * s2 * s;
  double ddpoly = 2 * 0.1260 + 12 * 0.3516 * s2 - 30 * 0.2843 * s2 * s2 +
                  56 * 0.1036 * s2 * s2 * s2;
  (void)as;
  X[1] = 5.0 * t * (0.2969 * s - sg * poly);
  D1[0] = 2.0 * s;
  D1[1] = 5.0 * t * (0.2969 - sg * dpoly);
  D2[0] = 2.0;
  D2[1] = 5.0 * t * (-sg * ddpoly);
}

static void airfoil_to_body(const orc_shape* s, const double x[2], double b[2]) {
  /* body frame: leading edge at origin, chord along +x, unit chord.  The
   * body is pitched nose-up by `incidence`: world = R(-a) body * chord + c. */
  double ca = cos(s->incidence), sa = sin(s->incidence);
  double dx = (x[0] - s->c[0]) / s->chord, dy = (x[1] - s->c[1]) / s->chord;
  /* inverse of rotation by -a is rotation by +a */
  b[0] = ca * dx - sa * dy;
  b[1] = sa * dx + ca * dy;
}

static void airfoil_to_world_vec(const orc_shape* s, const double b[2],
                                 double w[2]) {
  double ca = cos(s->incidence), sa = sin(s->incidence);
  w[0] = ca * b[0] + sa * b[1];
  w[1] = -sa * b[0] + ca * b[1];
}

static int airfoil_inside(const orc_shape* s, const double x[2], double* q) {
  double b[2];
  airfoil_to_body(s, x, b);
  if (b[0] < 0.0 || b[0] > 1.0) {
    *q = -fmin(fabs(b[0]), fabs(b[0] - 1.0)) - fabs(b[1]);
    return 0;
  }
  double yt = naca_yt(s->thick, b[0]);
  *q = (yt - fabs(b[1])) * s->chord;
  return fabs(b[1]) <= yt;
}

/* ------------------------------------------------------------------------- */
/* inside test and closest-point projection (Sec. 3.1)                      */
/* ------------------------------------------------------------------------- */

/* Returns 1 for a solid centre (psi >= 0), and the signed radial margin in q. */
static int inside_q(const orc_shape* s, int dim, const double* x, double* q) {
  double v[3] = {0, 0, 0}, rho2 = 0.0;
  if (s->kind == ORC_AIRFOIL) {
    if (dim != 2) { *q = 0; return 0; }
    return airfoil_inside(s, x, q);
  }
  for (int i = 0; i < dim; ++i) { v[i] = x[i] - s->c[i]; }
  for (int i = 0; i < dim; ++i) rho2 += v[i] * v[i];
  double rho = sqrt(rho2);
  double r;
  if (s->kind == ORC_SPHERE) {
    r = s->r0;
  } else if (s->kind == ORC_STAR2D) {
    if (rho == 0.0) { *q = s->r0; return 1; }
    double r1, r2;
    star_radius(s, atan2(v[1], v[0]), &r, &r1, &r2);
  } else {
    if (rho == 0.0) { *q = s->r0; return 1; }
    /* |Y_lm| <= 1 for Schmidt semi-normalised harmonics, so r lies within
     * r0 (1 -+ sum |a_lm|): far cells are settled without evaluating r */
    double sa = 0.0;
    for (int i = 0; i < s->ncoef; ++i) sa += fabs(s->coef[i]);
    double rmax = s->r0 * (1.0 + sa), rmin = s->r0 * (1.0 - sa);
    if (rho > rmax) { *q = rmax - rho; return 0; }
    if (rho < rmin) { *q = rmin - rho; return 1; }
    r = shstar_radius_value(s, v);
  }
  *q = r - rho;
  return *q >= 0.0;
}

int orc_shape_inside(const orc_shape* s, int dim, const double* x) {
  double q;
  return inside_q(s, dim, x, &q);
}

double orc_shape_radius(const orc_shape* s, int dim, const double* omega) {
  if (s->kind == ORC_SPHERE) return s->r0;
  if (s->kind == ORC_STAR2D) {
    double r, r1, r2;
    star_radius(s, atan2(omega[1], omega[0]), &r, &r1, &r2);
    return r;
  }
  if (s->kind == ORC_SHSTAR) {
    double v[3] = {omega[0], omega[1], dim == 3 ? omega[2] : 0.0};
    return shstar_radius(s, v).v;
  }
  return 0.0;
}

static void normalize(double* v, int dim) {
  double n = 0.0;
  for (int i = 0; i < dim; ++i) n += v[i] * v[i];
  n = sqrt(n);
  for (int i = 0; i < dim; ++i) v[i] /= n;
}

/* Closest boundary point S of x, outward unit normal n at S (analytic), and
 * psi = +|x - S| for solid centres, -|x - S| for fluid ones
 * (Eq. signed_distance).  Returns ORC_E_GEOMETRY if the iteration fails.   */
int orc_shape_project(const orc_shape* s, int dim, const double* x, int solid,
                      double* S, double* n, double* psi) {
  double v[3] = {0, 0, 0};
  for (int i = 0; i < dim; ++i) v[i] = x[i] - s->c[i];
  if (s->kind == ORC_SPHERE) {
    double rho2 = 0.0;
    for (int i = 0; i < dim; ++i) rho2 += v[i] * v[i];
    double rho = sqrt(rho2);
    if (rho == 0.0) return ORC_E_GEOMETRY;
    for (int i = 0; i < dim; ++i) n[i] = v[i] / rho;
    *psi = s->r0 - rho;
    for (int i = 0; i < dim; ++i) S[i] = s->c[i] + s->r0 * n[i];
    return ORC_OK;
  }
  if (s->kind == ORC_STAR2D) {
    /* Newton on theta for the stationarity of |X(theta) - x|^2 */
    double th = atan2(v[1], v[0]);
    int done = 0, extra = 0;
    for (int it = 0; it < 100; ++it) {
      double r, r1, r2;
      star_radius(s, th, &r, &r1, &r2);
      double ct = cos(th), st = sin(th);
      double X[2] = {s->c[0] + r * ct, s->c[1] + r * st};
      double D1[2] = {r1 * ct - r * st, r1 * st + r * ct};
      double D2[2] = {(r2 - r) * ct - 2.0 * r1 * st, (r2 - r) * st + 2.0 * r1 * ct};
      double R[2] = {X[0] - x[0], X[1] - x[1]};
      double g1 = R[0] * D1[0] + R[1] * D1[1];
      double g2 = D1[0] * D1[0] + D1[1] * D1[1] + R[0] * D2[0] + R[1] * D2[1];
      if (!(g2 > 0.0)) g2 = D1[0] * D1[0] + D1[1] * D1[1];
      double dth = -g1 / g2;
      th += dth;
      if (done) { if (++extra >= 2) break; }
      else if (fabs(dth) < 1e-13) done = 1;
    }
    if (!done) return ORC_E_GEOMETRY;
    double r, r1, r2;
    star_radius(s, th, &r, &r1, &r2);
    double ct = cos(th), st = sin(th);
    S[0] = s->c[0] + r * ct; S[1] = s->c[1] + r * st;
    double T[2] = {r1 * ct - r * st, r1 * st + r * ct};
    n[0] = T[1]; n[1] = -T[0];
    normalize(n, 2);
  } else if (s->kind == ORC_SHSTAR) {
    /* Gauss-Newton on the unit sphere of directions, tangent chart re-centred
     * at every iterate: S(omega) = c + r(omega) omega.                     */
    double om[3] = {v[0], v[1], v[2]};
    normalize(om, 3);
    int done = 0, extra = 0;
    for (int it = 0; it < 200; ++it) {
      dual rr = shstar_radius(s, om);
      double r = rr.v;
      /* tangent basis */
      int ax = 0;
      double am = fabs(om[0]);
      if (fabs(om[1]) < am) { ax = 1; am = fabs(om[1]); }
      if (fabs(om[2]) < am) { ax = 2; }
      double t1[3] = {0, 0, 0};
      t1[ax] = 1.0;
      double dt = t1[0] * om[0] + t1[1] * om[1] + t1[2] * om[2];
      for (int i = 0; i < 3; ++i) t1[i] -= dt * om[i];
      normalize(t1, 3);
      double t2[3] = {om[1] * t1[2] - om[2] * t1[1], om[2] * t1[0] - om[0] * t1[2],
                      om[0] * t1[1] - om[1] * t1[0]};
      double g1 = rr.d[0] * t1[0] + rr.d[1] * t1[1] + rr.d[2] * t1[2];
      double g2 = rr.d[0] * t2[0] + rr.d[1] * t2[1] + rr.d[2] * t2[2];
      double J1[3], J2[3], R[3];
      for (int i = 0; i < 3; ++i) {
        J1[i] = g1 * om[i] + r * t1[i];
        J2[i] = g2 * om[i] + r * t2[i];
        R[i] = s->c[i] + r * om[i] - x[i];
      }
      double a11 = 0, a12 = 0, a22 = 0, b1 = 0, b2 = 0;
      for (int i = 0; i < 3; ++i) {
        a11 += J1[i] * J1[i]; a12 += J1[i] * J2[i]; a22 += J2[i] * J2[i];
        b1 -= J1[i] * R[i]; b2 -= J2[i] * R[i];
      }
      double det = a11 * a22 - a12 * a12;
      double d1 = (b1 * a22 - b2 * a12) / det;
      double d2 = (a11 * b2 - a12 * b1) / det;
      for (int i = 0; i < 3; ++i) om[i] += d1 * t1[i] + d2 * t2[i];
      normalize(om, 3);
      if (done) { if (++extra >= 2) break; }
      else if (fabs(d1) + fabs(d2) < 1e-13) done = 1;
    }
    if (!done) return ORC_E_GEOMETRY;
    dual rr = shstar_radius(s, om);
    for (int i = 0; i < 3; ++i) {
      S[i] = s->c[i] + rr.v * om[i];
      /* outward normal of F(y) = |y - c| - r((y-c)/|y-c|): omega - grad r / r */
      n[i] = om[i] - rr.d[i] / rr.v;
    }
    normalize(n, 3);
  } else if (s->kind == ORC_AIRFOIL) {
    if (dim != 2) return ORC_E_UNSUPPORTED;
    double b[2];
    airfoil_to_body(s, x, b);
    /* start: the chord station of x, branch by side */
    double xc = b[0] < 0 ? 0 : (b[0] > 1 ? 1 : b[0]);
    double sp = sqrt(xc);
    double best_d2 = -1.0, best_s = 0.0;
    /* Newton from both branches; keep the nearer stationary/end point.     */
    double starts[2] = {sp, -sp};
    for (int st_i = 0; st_i < 2; ++st_i) {
      double sv = starts[st_i];
      if (sv == 0.0) sv = (st_i == 0) ? 1e-3 : -1e-3;
      double lo = st_i == 0 ? 0.0 : -1.0, hi = st_i == 0 ? 1.0 : 0.0;
      for (int it = 0; it < 100; ++it) {
        double X[2], D1[2], D2[2];
        naca_curve(s->thick, sv, X, D1, D2);
        double R[2] = {X[0] - b[0], X[1] - b[1]};
        double g1 = R[0] * D1[0] + R[1] * D1[1];
        double g2 = D1[0] * D1[0] + D1[1] * D1[1] + R[0] * D2[0] + R[1] * D2[1];
        if (!(g2 > 0.0)) g2 = D1[0] * D1[0] + D1[1] * D1[1];
        double ns = sv - g1 / g2;
        if (ns < lo) ns = lo;
        if (ns > hi) ns = hi;
        double ds = ns - sv;
        sv = ns;
        if (fabs(ds) < 1e-15) break;
      }
      double X[2], D1[2], D2[2];
      naca_curve(s->thick, sv, X, D1, D2);
      double d2 = (X[0] - b[0]) * (X[0] - b[0]) + (X[1] - b[1]) * (X[1] - b[1]);
      if (best_d2 < 0 || d2 < best_d2) { best_d2 = d2; best_s = sv; }
    }
    double X[2], D1[2], D2[2];
    naca_curve(s->thick, best_s, X, D1, D2);
    double nb[2];
    if (fabs(best_s) >= 1.0) {
      /* trailing-edge corner: direction from the corner to x */
      nb[0] = b[0] - X[0]; nb[1] = b[1] - X[1];
      if (solid) { nb[0] = -nb[0]; nb[1] = -nb[1]; }
    } else {
      /* the contour runs lower TE -> LE -> upper TE as s increases, i.e.
       * clockwise, so the outward normal is the tangent turned
       * counter-clockwise                                                  */
      nb[0] = -D1[1]; nb[1] = D1[0];
    }
    normalize(nb, 2);
    double w[2], Sb[2] = {X[0], X[1]}, Sw[2];
    airfoil_to_world_vec(s, nb, n);
    airfoil_to_world_vec(s, Sb, Sw);
    S[0] = s->c[0] + s->chord * Sw[0];
    S[1] = s->c[1] + s->chord * Sw[1];
    (void)w;
  } else {
    return ORC_E_UNSUPPORTED;
  }
  double d2 = 0.0;
  for (int i = 0; i < dim; ++i) d2 += (x[i] - S[i]) * (x[i] - S[i]);
  *psi = solid ? sqrt(d2) : -sqrt(d2);
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* plan                                                                      */
/* ------------------------------------------------------------------------- */

void orc_plan_destroy(orc_plan* p) {
  if (!p) return;
  free(p->coef); free(p->tag); free(p->lev_off); free(p->cell); free(p->level);
  free(p->delta); free(p->nrm); free(p->psi); free(p->r); free(p->e);
  free(p->sten); free(p->sorted_cell); free(p->sorted_pos);
  free(p->blk); free(p->blk_off); free(p->blk_mem);
  for (int i = 0; i < 3; ++i) free(p->faces[i]);
  free(p);
}

int orc_fresh_cells(const orc_plan* a, const orc_plan* b, int64_t* n_fresh,
                    int64_t* n_uncovered, int64_t* list, int64_t cap) {
  if (!a || !b || !n_fresh || !n_uncovered || a->dim != b->dim || a->ncell != b->ncell)
    return ORC_E_ARG;
  for (int i = 0; i < 3; ++i) if (a->g.n[i] != b->g.n[i]) return ORC_E_ARG;
  int64_t nf = 0, nu = 0;
  for (int64_t c = 0; c < a->ncell; ++c) {
    const int was_solid = a->tag[c] == 1 || a->tag[c] == 2;
    const int is_fluid = b->tag[c] == 0 || b->tag[c] == -2;
    if (!(was_solid && is_fluid)) continue;
    if (list && nf < cap) list[nf] = c;
    ++nf;
    if (a->tag[c] == 1) ++nu;
  }
  *n_fresh = nf;
  *n_uncovered = nu;
  return ORC_OK;
}

int64_t orc_n_cells(const orc_plan* p) { return p->ncell; }
int64_t orc_n_ghost(const orc_plan* p) { return p->ng; }
int64_t orc_n_interface(const orc_plan* p) { return p->nif; }
int32_t orc_n_levels(const orc_plan* p) { return p->nlev; }
int orc_dim(const orc_plan* p) { return p->dim; }

/* position of cell c among the linear-index-sorted ghosts, or -1 */
static int64_t find_ghost(const orc_plan* p, int64_t c) {
  int64_t lo = 0, hi = p->ng - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) / 2;
    if (p->sorted_cell[mid] == c) return p->sorted_pos[mid];
    if (p->sorted_cell[mid] < c) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

int orc_plan_create(const orc_grid* g, const orc_shape* s, int scheme,
                    orc_plan** out) {
  *out = NULL;
  if (!g || !s || (g->dim != 2 && g->dim != 3)) return ORC_E_ARG;
  /* scheme: CGC, CGC_ES or HGC, optionally with ORC_LAYER2 */
  const int layer2 = (scheme & ORC_LAYER2) != 0;
  scheme &= ~ORC_LAYER2;
  if (scheme < 0 || scheme > 2) return ORC_E_ARG;
  int dim = g->dim;
  for (int i = 0; i < dim; ++i) {
    if (g->n[i] < 1) return ORC_E_ARG;
    if (g->faces[i]) {
      for (int64_t k = 0; k < g->n[i]; ++k)
        if (!(g->faces[i][k + 1] > g->faces[i][k]) || !isfinite(g->faces[i][k + 1]))
          return ORC_E_ARG;
    } else if (!(g->h[i] > 0.0)) {
      return ORC_E_ARG;
    }
  }
  if (s->kind == ORC_SHSTAR && dim != 3) return ORC_E_ARG;
  if ((s->kind == ORC_STAR2D || s->kind == ORC_AIRFOIL) && dim != 2) return ORC_E_ARG;

  orc_plan* p = (orc_plan*)calloc(1, sizeof(orc_plan));
  if (!p) return ORC_E_NOMEM;
  p->g = *g;
  if (dim == 2) { p->g.n[2] = 1; p->g.lo[2] = 0.0; p->g.h[2] = 1.0; p->g.faces[2] = NULL; }
  for (int i = 0; i < dim; ++i) {
    p->faces[i] = NULL;
    if (!g->faces[i]) continue;
    p->faces[i] = (double*)malloc(sizeof(double) * (g->n[i] + 1));
    if (!p->faces[i]) { orc_plan_destroy(p); return ORC_E_NOMEM; }
    memcpy(p->faces[i], g->faces[i], sizeof(double) * (g->n[i] + 1));
    p->g.faces[i] = p->faces[i];
    p->g.lo[i] = p->faces[i][0];
  }
  p->s = *s;
  if (s->ncoef > 0) {
    int nc = (s->kind == ORC_STAR2D) ? 2 * s->ncoef : s->ncoef;
    p->coef = (double*)malloc(sizeof(double) * nc);
    memcpy(p->coef, s->coef, sizeof(double) * nc);
    p->s.coef = p->coef;
  }
  p->scheme = scheme;
  p->dim = dim;
  const orc_grid* G = &p->g;
  int64_t N = G->n[0] * G->n[1] * G->n[2];
  p->ncell = N;
  for (int i = 0; i < 7; ++i) p->margins[i] = (i >= 4) ? 0.0 : INFINITY;
  double hmin = INFINITY;   /* smallest cell width: the unit of the margins */
  for (int i = 0; i < dim; ++i)
    for (int64_t k = 0; k < (G->faces[i] ? G->n[i] : 1); ++k)
      if (width(G, i, k) < hmin) hmin = width(G, i, k);

  /* 1. classification by cell centre: fluid 0, solid 1 (Sec. 3.1) */
  uint8_t* solid = (uint8_t*)malloc(N);
  p->tag = (int8_t*)malloc(N);
  double* qm = (double*)malloc(sizeof(double) * N);
  if (!solid || !p->tag || !qm) { free(solid); free(qm); orc_plan_destroy(p); return ORC_E_NOMEM; }
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < N; ++c) {
    int64_t ijk[3];
    unlinear(G, c, ijk);
    double x[3] = {centre(G, 0, ijk[0]), centre(G, 1, ijk[1]),
                   dim == 3 ? centre(G, 2, ijk[2]) : 0.0};
    double q;
    solid[c] = (uint8_t)inside_q(&p->s, dim, x, &q);
    qm[c] = fabs(q) / hmin;
  }
  for (int64_t c = 0; c < N; ++c) {
    p->tag[c] = (int8_t)solid[c];
    if (qm[c] < p->margins[0]) p->margins[0] = qm[c];
  }
  free(qm);

  /* 2. cells with a face neighbour of the other class.  Both the CGC rule
   * ("solid cells immediately adjacent to the boundary") and the HGC rule
   * (candidates without an opposite face neighbour are reclassified) only
   * ever keep such cells, so the distance test is evaluated on them alone. */
  int64_t nif = 0;
  uint8_t* iface = (uint8_t*)calloc(N, 1);
  for (int64_t c = 0; c < N; ++c) {
    int64_t ijk[3];
    unlinear(G, c, ijk);
    for (int ax = 0; ax < dim && !iface[c]; ++ax)
      for (int sg = -1; sg <= 1; sg += 2) {
        int64_t nb[3] = {ijk[0], ijk[1], ijk[2]};
        nb[ax] += sg;
        if (nb[ax] < 0 || nb[ax] >= G->n[ax]) continue;
        if (solid[linear(G, nb)] != solid[c]) { iface[c] = 1; break; }
      }
    nif += iface[c];
  }
  p->nif = nif;
  /* Sec. 7.1 (additional ghost-cell layers): with a second layer, solid
   * cells with psi <= 1.5 delta n join the ghosts.  Candidates (value 2
   * here) are the solid cells with a fluid cell within R_i cells along each
   * axis i: going from x_c through its foot point S by a further half cell
   * diagonal reaches a point whose cell has a fluid centre (psi is
   * 1-Lipschitz), at most (1.5 + sqrt(d)/2) w_max away from x_c since
   * delta n <= w_max, the largest cell width of the grid; a displacement D
   * along axis i crosses at most floor(D / w_min_i) + 1 cells, w_min_i the
   * smallest width along i; hence R_i = floor((1.5 + sqrt(d)/2) w_max /
   * w_min_i) + 1 (h_max / h_i on a uniform grid).  Their distance to the
   * boundary decides below. */
  int64_t ncand = nif;
  if (layer2) {
    double wmax = 0.0, wmin[3] = {INFINITY, INFINITY, INFINITY};
    for (int i = 0; i < dim; ++i)
      for (int64_t k = 0; k < (G->faces[i] ? G->n[i] : 1); ++k) {
        const double w = width(G, i, k);
        if (w > wmax) wmax = w;
        if (w < wmin[i]) wmin[i] = w;
      }
    int64_t R[3] = {0, 0, 0};
    for (int i = 0; i < dim; ++i)
      R[i] = (int64_t)floor((1.5 + 0.5 * sqrt((double)dim)) * wmax / wmin[i]) + 1;
    for (int64_t c = 0; c < N; ++c) {
      if (!solid[c] || iface[c]) continue;
      int64_t ijk[3];
      unlinear(G, c, ijk);
      int found = 0;
      for (int64_t dk = -R[2]; dk <= R[2] && !found; ++dk)
        for (int64_t dj = -R[1]; dj <= R[1] && !found; ++dj)
          for (int64_t di = -R[0]; di <= R[0] && !found; ++di) {
            int64_t q[3] = {ijk[0] + di, ijk[1] + dj, ijk[2] + dk};
            int in = 1;
            for (int i = 0; i < 3; ++i) if (q[i] < 0 || q[i] >= G->n[i]) in = 0;
            if (in && !solid[linear(G, q)]) found = 1;
          }
      if (found) { iface[c] = 2; ++ncand; }
    }
  }

  /* 3. geometry and ghost tags on those cells */
  int64_t* ic = (int64_t*)malloc(sizeof(int64_t) * (ncand ? ncand : 1));
  double* igeo = (double*)malloc(sizeof(double) * 7 * (ncand ? ncand : 1));
  uint8_t* iext = (uint8_t*)calloc(ncand ? ncand : 1, 1);   /* second-layer ghost */
  int status = ORC_OK;
  {
    int64_t k = 0;
    for (int64_t c = 0; c < N; ++c) if (iface[c]) ic[k++] = c;
  }
  for (int64_t k = 0; k < ncand; ++k) {
    int64_t c = ic[k], ijk[3];
    unlinear(G, c, ijk);
    double x[3] = {centre(G, 0, ijk[0]), centre(G, 1, ijk[1]),
                   dim == 3 ? centre(G, 2, ijk[2]) : 0.0};
    double S[3] = {0, 0, 0}, n[3] = {0, 0, 0}, psi = 0.0;
    int st = orc_shape_project(&p->s, dim, x, solid[c], S, n, &psi);
    if (st != ORC_OK) { status = st; break; }
    /* Eq. delta_n, with the cell's own widths */
    double sum = 0.0;
    for (int i = 0; i < dim; ++i) {
      const double w = width(G, i, ijk[i]);
      sum += (n[i] / w) * (n[i] / w);
    }
    double dn = 1.0 / sqrt(sum);
    int8_t t = (int8_t)solid[c];
    if (scheme == ORC_HGC) {
      /* Eq. HGC_criterion, with reclassification (R1: judged on centres) */
      if (solid[c]) {
        if (psi <= dn / 2.0) t = 2;
        double m = fabs(psi - dn / 2.0) / hmin;
        if (m < p->margins[1]) p->margins[1] = m;
      } else {
        if (-psi < dn / 2.0) t = -2;
        double m = fabs(-psi - dn / 2.0) / hmin;
        if (m < p->margins[1]) p->margins[1] = m;
      }
    } else {
      /* CGC / CGC_ES: solid cells with a fluid face neighbour */
      if (solid[c] && iface[c] == 1) t = 2;
    }
    if (layer2 && solid[c] && t != 2) {
      /* second layer: solid cells with psi <= 1.5 delta n, on the extended
       * stencil of Eq. stencil_anisotropic */
      if (psi <= 1.5 * dn) { t = 2; iext[k] = 1; }
      double m = fabs(psi - 1.5 * dn) / hmin;
      if (m < p->margins[1]) p->margins[1] = m;
    }
    p->tag[c] = t;
    igeo[7 * k + 0] = psi;
    for (int i = 0; i < 3; ++i) { igeo[7 * k + 1 + i] = n[i]; }
    for (int i = 0; i < 3; ++i) { igeo[7 * k + 4 + i] = S[i]; }
  }
  if (status != ORC_OK) {
    free(solid); free(iface); free(ic); free(igeo); free(iext); orc_plan_destroy(p);
    return status;
  }

  /* 4. ghost list in linear-index order */
  int64_t ng = 0;
  for (int64_t k = 0; k < ncand; ++k) if (p->tag[ic[k]] == 2 || p->tag[ic[k]] == -2) ++ng;
  p->ng = ng;
  int64_t na = ng ? ng : 1;
  int64_t* gcell = (int64_t*)malloc(sizeof(int64_t) * na);
  double* gpsi = (double*)malloc(sizeof(double) * na);
  double* gn = (double*)malloc(sizeof(double) * 3 * na);
  uint8_t* gext = (uint8_t*)calloc(na, 1);
  {
    int64_t j = 0;
    for (int64_t k = 0; k < ncand; ++k) {
      int8_t t = p->tag[ic[k]];
      if (t != 2 && t != -2) continue;
      gcell[j] = ic[k];
      gext[j] = iext[k];
      gpsi[j] = igeo[7 * k];
      for (int i = 0; i < 3; ++i) gn[3 * j + i] = igeo[7 * k + 1 + i];
      ++j;
    }
  }
  free(ic); free(igeo); free(iext);

  /* 5. stencil per ghost: e = sgn(n) with sgn(0) = +1 (Appendix A), r_i = 1
   * or Eq. stencil_anisotropic (CGC_ES), x_s = x_c + psi n (Eq.
   * signed_distance: S lies on the normal through x_c at distance |psi|). */
  int np = npts(dim);
  int32_t* ge = (int32_t*)malloc(sizeof(int32_t) * 3 * na);
  int32_t* gr = (int32_t*)malloc(sizeof(int32_t) * 3 * na);
  double* gd = (double*)malloc(sizeof(double) * 3 * na);
  int64_t* gst = (int64_t*)malloc(sizeof(int64_t) * 7 * na);
  int64_t* dep = (int64_t*)malloc(sizeof(int64_t) * 7 * na); /* linear-order ghost ids */
  for (int64_t j = 0; j < ng; ++j) {
    int64_t ijk[3];
    unlinear(G, gcell[j], ijk);
    for (int i = 0; i < 3; ++i) {
      double ni = gn[3 * j + i];
      gd[3 * j + i] = gpsi[j] * ni;
      ge[3 * j + i] = (ni >= 0.0) ? 1 : -1;
      gr[3 * j + i] = 1;
      if (i < dim && ni != 0.0 && fabs(ni) < p->margins[3]) p->margins[3] = fabs(ni);
    }
    if (scheme == ORC_CGC_ES || gext[j]) {
      for (int i = 0; i < dim; ++i) {
        double q = 2.0 * fabs(gd[3 * j + i]) / width(G, i, ijk[i]);
        int ri = (int)ceil(q);
        if (ri < 1) ri = 1;
        gr[3 * j + i] = ri;
        double nearest = floor(q + 0.5);
        if (nearest < 1.0) nearest = 1.0;
        double m = fabs(q - nearest);
        if (m < p->margins[2]) p->margins[2] = m;
      }
    }
    for (int k = 0; k < np; ++k) {
      const int* sb = subset(dim, k);
      int skip = 0;
      int64_t q[3] = {ijk[0], ijk[1], ijk[2]};
      for (int i = 0; i < dim; ++i)
        if (sb[i]) {
          if (gn[3 * j + i] == 0.0) skip = 1;
          q[i] += (int64_t)ge[3 * j + i] * gr[3 * j + i];
        }
      gst[7 * j + k] = -1;
      dep[7 * j + k] = -1;
      if (skip) continue;
      for (int i = 0; i < dim; ++i)
        if (q[i] < 0 || q[i] >= G->n[i]) status = ORC_E_STENCIL;
      if (status != ORC_OK) break;
      int64_t qc = linear(G, q);
      if (p->tag[qc] == 1) { status = ORC_E_STENCIL; break; }
      gst[7 * j + k] = qc;
      if (p->tag[qc] == 2 || p->tag[qc] == -2) {
        /* ghost-to-ghost edge (Sec. 3.2) */
        int64_t lo = 0, hi = ng - 1, f = -1;
        while (lo <= hi) {
          int64_t mid = (lo + hi) / 2;
          if (gcell[mid] == qc) { f = mid; break; }
          if (gcell[mid] < qc) lo = mid + 1; else hi = mid - 1;
        }
        dep[7 * j + k] = f;
      }
    }
    if (status != ORC_OK) break;
  }

  /* 6. Levels (Sec. 3.2).  Kahn's layering: L1 = units whose stencils hold
   * no ghost outside the unit; a unit joins L_k once every ghost it needs
   * lies in L_1..L_{k-1}.  A unit is a single ghost, except where the
   * dependency graph is not acyclic (the paper asserts acyclicity; two
   * ghosts at the bottom of a concave valley whose normals lean towards each
   * other read each other): each strongly connected component (Tarjan) is
   * one unit whose coupled relations are solved together, which is the
   * fixed point an iterative reconstruction converges to.               */
  int32_t* lev = (int32_t*)calloc(na, sizeof(int32_t));
  int64_t* order = (int64_t*)malloc(sizeof(int64_t) * na);
  int64_t* comp = (int64_t*)malloc(sizeof(int64_t) * na);
  int32_t* lev_off = NULL;
  int32_t nlev = 0;
  int64_t ncomp = 0;
  if (status == ORC_OK) {
    /* Tarjan, iterative */
    int64_t* tidx = (int64_t*)malloc(sizeof(int64_t) * na);
    int64_t* tlow = (int64_t*)malloc(sizeof(int64_t) * na);
    int64_t* stk = (int64_t*)malloc(sizeof(int64_t) * na);
    int64_t* cs = (int64_t*)malloc(sizeof(int64_t) * na);
    int32_t* cit = (int32_t*)malloc(sizeof(int32_t) * na);
    uint8_t* onst = (uint8_t*)calloc(na, 1);
    int64_t counter = 0, sp = 0;
    for (int64_t j = 0; j < ng; ++j) tidx[j] = -1;
    for (int64_t root = 0; root < ng; ++root) {
      if (tidx[root] >= 0) continue;
      int64_t csp = 0;
      cs[csp] = root; cit[csp] = 0; ++csp;
      tidx[root] = tlow[root] = counter++;
      stk[sp++] = root; onst[root] = 1;
      while (csp > 0) {
        int64_t v = cs[csp - 1];
        if (cit[csp - 1] < np) {
          int64_t w = dep[7 * v + cit[csp - 1]];
          cit[csp - 1]++;
          if (w < 0) continue;
          if (tidx[w] < 0) {
            tidx[w] = tlow[w] = counter++;
            stk[sp++] = w; onst[w] = 1;
            cs[csp] = w; cit[csp] = 0; ++csp;
          } else if (onst[w] && tidx[w] < tlow[v]) {
            tlow[v] = tidx[w];
          }
        } else {
          if (tlow[v] == tidx[v]) {
            int64_t x;
            do { x = stk[--sp]; onst[x] = 0; comp[x] = ncomp; } while (x != v);
            ++ncomp;
          }
          --csp;
          if (csp > 0 && tlow[v] < tlow[cs[csp - 1]]) tlow[cs[csp - 1]] = tlow[v];
        }
      }
    }
    free(tidx); free(tlow); free(stk); free(cs); free(cit); free(onst);
    int64_t* csize = (int64_t*)calloc(ncomp ? ncomp : 1, sizeof(int64_t));
    for (int64_t j = 0; j < ng; ++j) csize[comp[j]]++;
    for (int64_t u = 0; u < ncomp; ++u)
      if (csize[u] > 1) { p->nblk++; if (csize[u] > p->maxblk) p->maxblk = (int32_t)csize[u]; }
    free(csize);
    if (status == ORC_OK) {
      /* Kahn on the condensed graph */
      int64_t nu = ncomp ? ncomp : 1;
      int32_t* indeg = (int32_t*)calloc(nu, sizeof(int32_t));
      int64_t* rd_off = (int64_t*)calloc(nu + 1, sizeof(int64_t));
      for (int64_t j = 0; j < ng; ++j)
        for (int k = 0; k < np; ++k) {
          int64_t d = dep[7 * j + k];
          if (d >= 0 && comp[d] != comp[j]) { indeg[comp[j]]++; rd_off[comp[d] + 1]++; }
        }
      for (int64_t u = 0; u < ncomp; ++u) rd_off[u + 1] += rd_off[u];
      int64_t* rd = (int64_t*)malloc(sizeof(int64_t) * (rd_off[ncomp] ? rd_off[ncomp] : 1));
      int64_t* fillp = (int64_t*)malloc(sizeof(int64_t) * nu);
      for (int64_t u = 0; u < ncomp; ++u) fillp[u] = rd_off[u];
      for (int64_t j = 0; j < ng; ++j)
        for (int k = 0; k < np; ++k) {
          int64_t d = dep[7 * j + k];
          if (d >= 0 && comp[d] != comp[j]) rd[fillp[comp[d]]++] = comp[j];
        }
      free(fillp);
      int32_t* ulev = (int32_t*)calloc(nu, sizeof(int32_t));
      int64_t* uq = (int64_t*)malloc(sizeof(int64_t) * nu);
      int64_t head = 0, tail = 0;
      for (int64_t u = 0; u < ncomp; ++u)
        if (indeg[u] == 0) { uq[tail++] = u; ulev[u] = 1; }
      while (head < tail) {
        int64_t end = tail;
        ++nlev;
        for (; head < end; ++head) {
          int64_t u = uq[head];
          for (int64_t t = rd_off[u]; t < rd_off[u + 1]; ++t) {
            int64_t w = rd[t];
            if (--indeg[w] == 0) { uq[tail++] = w; ulev[w] = nlev + 1; }
          }
        }
      }
      if (tail != ncomp) status = ORC_E_CYCLE;   /* cannot happen on a condensation */
      for (int64_t j = 0; j < ng; ++j) lev[j] = ulev[comp[j]];
      free(indeg); free(rd_off); free(rd); free(ulev); free(uq);
      /* ghosts by level, linear index ascending inside a level */
      lev_off = (int32_t*)calloc(nlev + 2, sizeof(int32_t));
      for (int64_t j = 0; j < ng; ++j) lev_off[lev[j]]++;
      for (int32_t l = 1; l <= nlev; ++l) lev_off[l] += lev_off[l - 1];
      int32_t* put = (int32_t*)malloc(sizeof(int32_t) * (nlev + 1));
      for (int32_t l = 0; l <= nlev; ++l) put[l] = lev_off[l];
      for (int64_t j = 0; j < ng; ++j) order[put[lev[j] - 1]++] = j;
      free(put);
    }
  }

  if (status != ORC_OK) {
    free(solid); free(iface); free(gcell); free(gpsi); free(gn); free(gext); free(ge); free(gr);
    free(gd); free(gst); free(dep); free(lev); free(order); free(lev_off); free(comp);
    orc_plan_destroy(p);
    return status;
  }

  /* 7. canonical order: level ascending, linear index ascending inside a
   * level (units of a level are independent, so any order is valid).  Ids
   * follow the linear index, and the bucketing above kept id order.      */
  p->nlev = nlev;
  p->lev_off = (int32_t*)malloc(sizeof(int32_t) * (nlev + 1));
  memcpy(p->lev_off, lev_off, sizeof(int32_t) * (nlev + 1));
  p->cell = (int64_t*)malloc(sizeof(int64_t) * na);
  p->level = (int32_t*)malloc(sizeof(int32_t) * na);
  p->delta = (double*)calloc(3 * na, sizeof(double));
  p->nrm = (double*)calloc(3 * na, sizeof(double));
  p->psi = (double*)malloc(sizeof(double) * na);
  p->r = (int32_t*)malloc(sizeof(int32_t) * 3 * na);
  p->e = (int32_t*)malloc(sizeof(int32_t) * 3 * na);
  p->sten = (int64_t*)malloc(sizeof(int64_t) * 7 * na);
  p->sorted_cell = (int64_t*)malloc(sizeof(int64_t) * na);
  p->sorted_pos = (int64_t*)malloc(sizeof(int64_t) * na);
  for (int64_t pos = 0; pos < ng; ++pos) {
    int64_t j = order[pos];
    p->cell[pos] = gcell[j];
    p->level[pos] = lev[j];
    p->psi[pos] = gpsi[j];
    for (int i = 0; i < 3; ++i) {
      p->delta[i * ng + pos] = gd[3 * j + i];
      p->nrm[i * ng + pos] = gn[3 * j + i];
      p->r[i * ng + pos] = gr[3 * j + i];
      p->e[i * ng + pos] = ge[3 * j + i];
    }
    for (int k = 0; k < 7; ++k) p->sten[7 * pos + k] = gst[7 * j + k];
    p->sorted_cell[j] = gcell[j];
    p->sorted_pos[j] = pos;
    /* normalised boundary distance alpha_i = (x_s - x_1)/(x_2 - x_1) */
    {
      int64_t ijk[3];
      unlinear(G, gcell[j], ijk);
      for (int i = 0; i < dim; ++i) {
        double a = gd[3 * j + i] / span(G, i, ijk[i], ge[3 * j + i] * gr[3 * j + i]);
        if (a > p->margins[4 + i]) p->margins[4 + i] = a;
      }
    }
  }
  /* coupled units: members in canonical order */
  p->blk = (int32_t*)malloc(sizeof(int32_t) * na);
  p->blk_off = (int32_t*)calloc(p->nblk + 1, sizeof(int32_t));
  p->blk_mem = (int64_t*)malloc(sizeof(int64_t) * (ng ? ng : 1));
  {
    int64_t* cid = (int64_t*)malloc(sizeof(int64_t) * (ncomp ? ncomp : 1));
    int64_t* csz = (int64_t*)calloc(ncomp ? ncomp : 1, sizeof(int64_t));
    for (int64_t j = 0; j < ng; ++j) csz[comp[j]]++;
    int32_t nb = 0;
    for (int64_t u = 0; u < ncomp; ++u) cid[u] = (csz[u] > 1) ? nb++ : -1;
    for (int32_t b = 0; b < nb; ++b) p->blk_off[b + 1] = 0;
    for (int64_t u = 0; u < ncomp; ++u) if (cid[u] >= 0) p->blk_off[cid[u] + 1] = (int32_t)csz[u];
    for (int32_t b = 0; b < nb; ++b) p->blk_off[b + 1] += p->blk_off[b];
    int32_t* put = (int32_t*)malloc(sizeof(int32_t) * (nb + 1));
    for (int32_t b = 0; b <= nb; ++b) put[b] = p->blk_off[b];
    for (int64_t pos = 0; pos < ng; ++pos) {
      int64_t u = comp[order[pos]];
      p->blk[pos] = (int32_t)cid[u];
      if (cid[u] >= 0) p->blk_mem[put[cid[u]]++] = pos;
    }
    free(put); free(cid); free(csz);
  }
  free(solid); free(iface); free(gcell); free(gpsi); free(gn); free(gext); free(ge); free(gr);
  free(gd); free(gst); free(dep); free(lev); free(order); free(lev_off); free(comp);
  *out = p;
  return ORC_OK;
}

void orc_export(const orc_plan* p, int8_t* tags, int64_t* ghost_cell,
                int32_t* level_off, int32_t* level, double* delta,
                double* normal, double* psi, int32_t* r) {
  int64_t ng = p->ng;
  if (tags) memcpy(tags, p->tag, (size_t)p->ncell);
  if (ghost_cell) memcpy(ghost_cell, p->cell, sizeof(int64_t) * ng);
  if (level_off) memcpy(level_off, p->lev_off, sizeof(int32_t) * (p->nlev + 1));
  if (level) memcpy(level, p->level, sizeof(int32_t) * ng);
  if (psi) memcpy(psi, p->psi, sizeof(double) * ng);
  for (int i = 0; i < p->dim; ++i) {
    if (delta) memcpy(delta + i * ng, p->delta + i * ng, sizeof(double) * ng);
    if (normal) memcpy(normal + i * ng, p->nrm + i * ng, sizeof(double) * ng);
    if (r) memcpy(r + i * ng, p->r + i * ng, sizeof(int32_t) * ng);
  }
}

void orc_stencil(const orc_plan* p, int64_t g, int64_t* cells) {
  for (int k = 0; k < npts(p->dim); ++k) cells[k] = p->sten[7 * g + k];
}

void orc_units(const orc_plan* p, int32_t* nblk, int32_t* maxblk, int32_t* unit) {
  *nblk = p->nblk;
  *maxblk = p->maxblk;
  if (unit) memcpy(unit, p->blk, sizeof(int32_t) * p->ng);
}

void orc_margins(const orc_plan* p, double* out) {
  for (int i = 0; i < 7; ++i) out[i] = p->margins[i];
}

/* ------------------------------------------------------------------------- */
/* reconstruction weights (Sec. 4.1, Sec. 5.1)                               */
/* ------------------------------------------------------------------------- */

/* Coordinates relative to G (x_1 = 0): x_2 = r e dx, x_s = delta. */
static void local_coords(const orc_plan* p, int64_t g, double x2[3], double xs[3],
                         double n[3]) {
  int64_t ng = p->ng;
  int64_t ijk[3];
  unlinear(&p->g, p->cell[g], ijk);
  for (int i = 0; i < 3; ++i) {
    if (i < p->dim) {
      x2[i] = span(&p->g, i, ijk[i], p->e[i * ng + g] * p->r[i * ng + g]);
      xs[i] = p->delta[i * ng + g];
      n[i] = p->nrm[i * ng + g];
    } else {
      x2[i] = 1.0; xs[i] = 0.0; n[i] = 0.0;
    }
  }
}

/* Weights on P1..P(2^d-1) and on the boundary datum, in coordinates
 * relative to G (x_1 = 0): x2 = r e dx, xs = x_s - x_1, n = unit normal. */
int orc_weights_raw(int dim, int bc, const double* x2, const double* xs,
                    const double* n, double* w, double* ws) {
  const double x1 = 0.0, y1 = 0.0, z1 = 0.0;
  double X2 = x2[0], Y2 = x2[1], Z2 = dim == 3 ? x2[2] : 1.0;
  double Xs = xs[0], Ys = xs[1], Zs = dim == 3 ? xs[2] : 0.0;
  if (dim == 2) {
    if (bc == ORC_DIRICHLET) {
      /* Eq. phi_G_Dir_2d */
      double w1 = (x1 - Xs) / (X2 - Xs);
      double w2 = (y1 - Ys) / (Y2 - Ys);
      w[0] = w1; w[1] = w2; w[2] = -w1 * w2;
      *ws = (1.0 - w1) * (1.0 - w2);
    } else {
      /* Eq. phi_G_Neu_2d */
      double a1 = n[0] * (y1 - Ys), a2 = n[0] * (Y2 - Ys);
      double b1 = n[1] * (x1 - Xs), b2 = n[1] * (X2 - Xs);
      double w1 = (a2 + b1) / (a2 + b2);
      double w2 = (a1 + b2) / (a2 + b2);
      w[0] = w1; w[1] = w2; w[2] = 1.0 - w1 - w2;
      *ws = -(X2 - x1) * (Y2 - y1) / (a2 + b2);
    }
  } else {
    if (bc == ORC_DIRICHLET) {
      /* Eq. phi_G_Dir_3d */
      double w1 = (x1 - Xs) / (X2 - Xs);
      double w2 = (y1 - Ys) / (Y2 - Ys);
      double w3 = (z1 - Zs) / (Z2 - Zs);
      w[0] = w1; w[1] = w2; w[2] = w3;
      w[3] = -w1 * w2; w[4] = -w2 * w3; w[5] = -w1 * w3; w[6] = w1 * w2 * w3;
      *ws = (1.0 - w1) * (1.0 - w2) * (1.0 - w3);
    } else {
      /* Eq. phi_G_Neu_3d: a_ij = n_x (y_i - y_s)(z_j - z_s),
       * b_ij = n_y (x_i - x_s)(z_j - z_s), c_ij = n_z (x_i - x_s)(y_j - y_s) */
      double xv[3] = {0, x1 - Xs, X2 - Xs}, yv[3] = {0, y1 - Ys, Y2 - Ys},
             zv[3] = {0, z1 - Zs, Z2 - Zs};
#define A(i, j) (n[0] * yv[i] * zv[j])
#define B(i, j) (n[1] * xv[i] * zv[j])
#define C(i, j) (n[2] * xv[i] * yv[j])
      double D = A(2, 2) + B(2, 2) + C(2, 2);
      w[0] = (A(2, 2) + B(1, 2) + C(1, 2)) / D;
      w[1] = (A(1, 2) + B(2, 2) + C(2, 1)) / D;
      w[2] = (A(2, 1) + B(2, 1) + C(2, 2)) / D;
      w[3] = -(A(1, 2) + B(1, 2) + C(1, 1)) / D;
      w[4] = -(A(1, 1) + B(2, 1) + C(2, 1)) / D;
      w[5] = -(A(2, 1) + B(1, 1) + C(1, 2)) / D;
      w[6] = (A(1, 1) + B(1, 1) + C(1, 1)) / D;
      *ws = -(X2 - x1) * (Y2 - y1) * (Z2 - z1) / D;
#undef A
#undef B
#undef C
    }
  }
  return ORC_OK;
}

int orc_weights(const orc_plan* p, int64_t g, int bc, double* w, double* ws) {
  if (g < 0 || g >= p->ng) return ORC_E_ARG;
  double x2[3], xs[3], n[3];
  local_coords(p, g, x2, xs, n);
  return orc_weights_raw(p->dim, bc, x2, xs, n, w, ws);
}

/* Sensitivity bounds of the weights, for tolerances: wb[k] = |w_k| + sum_i
 * (|x2_i| |dw_k/dxs_i| + |dw_k/dn_i|), wsb likewise for w_s.  Each side of a
 * parity comparison computes the foot point and normal by its own
 * projection (Newton's method for star, spherical-harmonic and airfoil
 * bodies), so x_s and n agree to a small fraction of a cell and of a unit,
 * not bit for bit; a weight's scale is then how far it moves under a
 * perturbation of x_s on the scale of the stencil span and of n on the scale
 * of a unit vector.  Derivatives by central differences of the closed forms
 * with relative steps 1e-7 (their truncation error is far below what a
 * tolerance needs). */
int orc_weight_bounds_raw(int dim, int bc, const double* x2, const double* xs,
                          const double* n, double* wb, double* wsb) {
  const int np = npts(dim);
  double w[7], ws;
  orc_weights_raw(dim, bc, x2, xs, n, w, &ws);
  for (int k = 0; k < np; ++k) wb[k] = fabs(w[k]);
  *wsb = fabs(ws);
  for (int which = 0; which < 2; ++which) {
    for (int i = 0; i < dim; ++i) {
      double a[3] = {xs[0], xs[1], dim == 3 ? xs[2] : 0.0};
      double b[3] = {n[0], n[1], dim == 3 ? n[2] : 0.0};
      double* v = which == 0 ? a : b;
      const double scale = which == 0 ? fabs(x2[i]) : 1.0;
      const double eta = 1e-7 * scale;
      const double v0 = v[i];
      double wp[7], wsp, wm[7], wsm;
      v[i] = v0 + eta;
      orc_weights_raw(dim, bc, x2, a, b, wp, &wsp);
      v[i] = v0 - eta;
      orc_weights_raw(dim, bc, x2, a, b, wm, &wsm);
      for (int k = 0; k < np; ++k) wb[k] += scale * fabs((wp[k] - wm[k]) / (2.0 * eta));
      *wsb += scale * fabs((wsp - wsm) / (2.0 * eta));
    }
  }
  return ORC_OK;
}

int orc_weight_bounds(const orc_plan* p, int64_t g, int bc, double* wb, double* wsb) {
  if (g < 0 || g >= p->ng) return ORC_E_ARG;
  double x2[3], xs[3], n[3];
  local_coords(p, g, x2, xs, n);
  return orc_weight_bounds_raw(p->dim, bc, x2, xs, n, wb, wsb);
}

/* one ghost value from the current field values (skipped points not read) */
static double ghost_value(const orc_plan* p, int64_t g, const double* f, int bc,
                          double b) {
  double w[7], ws;
  orc_weights(p, g, bc, w, &ws);
  double v = 0.0;
  for (int k = 0; k < npts(p->dim); ++k) {
    int64_t c = p->sten[7 * g + k];
    if (c >= 0) v += w[k] * f[c];
  }
  return v + ws * b;
}

/* Gaussian elimination with partial pivoting: A (k x k, row major) x = b;
 * A and b are overwritten, x returned in b. */
static int gauss(int k, double* A, double* b) {
  for (int c = 0; c < k; ++c) {
    int piv = c;
    for (int r = c + 1; r < k; ++r) if (fabs(A[r * k + c]) > fabs(A[piv * k + c])) piv = r;
    if (A[piv * k + c] == 0.0) return ORC_E_DEGENERATE;
    if (piv != c) {
      for (int t = 0; t < k; ++t) { double x = A[c * k + t]; A[c * k + t] = A[piv * k + t]; A[piv * k + t] = x; }
      double x = b[c]; b[c] = b[piv]; b[piv] = x;
    }
    for (int r = c + 1; r < k; ++r) {
      double f = A[r * k + c] / A[c * k + c];
      for (int t = c; t < k; ++t) A[r * k + t] -= f * A[c * k + t];
      b[r] -= f * b[c];
    }
  }
  for (int c = k - 1; c >= 0; --c) {
    double v = b[c];
    for (int t = c + 1; t < k; ++t) v -= A[c * k + t] * b[t];
    b[c] = v / A[c * k + c];
  }
  return ORC_OK;
}

static int32_t unit_size(const orc_plan* p, int32_t u) {
  return p->blk_off[u + 1] - p->blk_off[u];
}

/* Coupled unit u: matrix A = I - (weights among members), and for member i
 * the external part rhs_i = sum_ext w f + w_s b (or its absolute-value
 * bound when `absval`, with f holding scales).  f == NULL: matrix only. */
static int unit_system(const orc_plan* p, int32_t u, const double* f,
                       const int8_t* bct, const double* bv, double* A,
                       double* rhs, int absval, const double* gscale) {
  int32_t k = p->blk_off[u + 1] - p->blk_off[u];
  const int64_t* m = p->blk_mem + p->blk_off[u];
  for (int i = 0; i < k * k; ++i) A[i] = 0.0;
  for (int i = 0; i < k; ++i) {
    double w[7], ws, wb[7], wsb;
    orc_weights(p, m[i], bct[m[i]], w, &ws);
    if (absval) orc_weight_bounds(p, m[i], bct[m[i]], wb, &wsb);
    A[i * k + i] = 1.0;
    rhs[i] = !bv ? 0.0 : (absval ? wsb * fabs(bv[m[i]]) : ws * bv[m[i]]);
    for (int j = 0; j < npts(p->dim); ++j) {
      int64_t c = p->sten[7 * m[i] + j];
      if (c < 0) continue;
      int t = -1;
      for (int q = 0; q < k; ++q) if (p->cell[m[q]] == c) t = q;
      if (t >= 0) { A[i * k + t] -= w[j]; continue; }
      if (!f) continue;
      if (!absval) rhs[i] += w[j] * f[c];
      else {
        double sv = (p->tag[c] == 2 || p->tag[c] == -2) ? gscale[find_ghost(p, c)] : fabs(f[c]);
        rhs[i] += wb[j] * sv;
      }
    }
  }
  return k;
}

int orc_fill(const orc_plan* p, int nf, double* fields, const int8_t* bc_type,
             const double* bc_val) {
  /* levels L1..Ln in order; each unit evaluated once (Sec. 3.2) */
  for (int f = 0; f < nf; ++f) {
    double* F = fields + (int64_t)f * p->ncell;
    const int8_t* bt = bc_type + (int64_t)f * p->ng;
    const double* bv = bc_val + (int64_t)f * p->ng;
    for (int64_t g = 0; g < p->ng; ++g) {
      int32_t u = p->blk[g];
      if (u < 0) {
        F[p->cell[g]] = ghost_value(p, g, F, bt[g], bv[g]);
      } else if (g == p->blk_mem[p->blk_off[u]]) {
        const int32_t k = unit_size(p, u);
        double* A = (double*)malloc(sizeof(double) * k * (k + 1));
        if (!A) return ORC_E_NOMEM;
        double* x = A + (int64_t)k * k;
        unit_system(p, u, F, bt, bv, A, x, 0, NULL);
        int st = gauss(k, A, x);
        if (st == ORC_OK)
          for (int i = 0; i < k; ++i) F[p->cell[p->blk_mem[p->blk_off[u] + i]]] = x[i];
        free(A);
        if (st != ORC_OK) return st;
      }
    }
  }
  return ORC_OK;
}

int orc_fill_jacobi(const orc_plan* p, int nf, double* fields,
                    const int8_t* bc_type, const double* bc_val, int max_sweeps) {
  /* synchronous sweeps: every ghost recomputed from the previous iterate */
  int64_t ng = p->ng;
  double* nv = (double*)malloc(sizeof(double) * (ng ? ng : 1));
  int result = -1;
  for (int f = 0; f < nf; ++f) {
    double* F = fields + (int64_t)f * p->ncell;
    for (int64_t g = 0; g < ng; ++g) F[p->cell[g]] = NAN;
    int done_at = -1;
    for (int s = 1; s <= max_sweeps; ++s) {
      int changed = 0;
      for (int64_t g = 0; g < ng; ++g) {
        int64_t k = (int64_t)f * ng + g;
        nv[g] = ghost_value(p, g, F, bc_type[k], bc_val[k]);
      }
      for (int64_t g = 0; g < ng; ++g) {
        double o = F[p->cell[g]];
        if (!(o == nv[g])) changed = 1; /* NaN counts as not yet final */
        F[p->cell[g]] = nv[g];
      }
      int finite = 1;
      for (int64_t g = 0; g < ng; ++g) if (isnan(nv[g])) { finite = 0; break; }
      if (!changed && finite) { done_at = s - 1; break; }
    }
    if (f == 0 || done_at > result) result = done_at;
    if (done_at < 0) { result = -1; break; }
  }
  free(nv);
  return result;
}

/* |A^-1| of coupled unit u (A from unit_system), row major k x k, column
 * by column from solves against unit vectors; NULL if out of memory. */
static double* unit_abs_inverse(const orc_plan* p, int32_t u, const int8_t* bct) {
  const int32_t k = unit_size(p, u);
  double* out = (double*)malloc(sizeof(double) * (2 * k * k + k));
  if (!out) return NULL;
  double* A = out + (int64_t)k * k;
  double* e = A + (int64_t)k * k;
  for (int t = 0; t < k; ++t) {
    unit_system(p, u, NULL, bct, NULL, A, e, 0, NULL);   /* gauss overwrites A */
    for (int q = 0; q < k; ++q) e[q] = (q == t) ? 1.0 : 0.0;
    gauss(k, A, e);
    for (int i = 0; i < k; ++i) out[i * k + t] = fabs(e[i]);
  }
  return out;
}

int orc_fill_scale(const orc_plan* p, int nf, const double* fields,
                   const int8_t* bc_type, const double* bc_val, double* scale) {
  /* s_G = sum_k wb_k s_{P_k} + wsb_G |b_G| with the weight bounds above
   * (|w| plus the weights' sensitivity to the geometry), s = |phi| on
   * non-ghost cells; coupled units: s = |A^-1| (external bound). */
  int64_t ng = p->ng;
  for (int f = 0; f < nf; ++f) {
    const double* F = fields + (int64_t)f * p->ncell;
    const int8_t* bt = bc_type + (int64_t)f * ng;
    const double* bv = bc_val + (int64_t)f * ng;
    double* sc = scale + (int64_t)f * ng;
    for (int64_t g = 0; g < ng; ++g) {
      int32_t u = p->blk[g];
      if (u >= 0) {
        if (g != p->blk_mem[p->blk_off[u]]) continue;
        const int32_t k = unit_size(p, u);
        double* inv = unit_abs_inverse(p, u, bt);
        double* A = (double*)malloc(sizeof(double) * k * (k + 1));
        if (!inv || !A) { free(inv); free(A); return ORC_E_NOMEM; }
        double* r = A + (int64_t)k * k;
        unit_system(p, u, F, bt, bv, A, r, 1, sc);
        for (int i = 0; i < k; ++i) {
          double acc = 0.0;
          for (int t = 0; t < k; ++t) acc += inv[i * k + t] * r[t];
          sc[p->blk_mem[p->blk_off[u] + i]] = acc;
        }
        free(inv); free(A);
        continue;
      }
      double wb[7], wsb;
      orc_weight_bounds(p, g, bt[g], wb, &wsb);
      double s = wsb * fabs(bv[g]);
      for (int j = 0; j < npts(p->dim); ++j) {
        int64_t c = p->sten[7 * g + j];
        if (c < 0) continue;
        double sv;
        if (p->tag[c] == 2 || p->tag[c] == -2) sv = sc[find_ghost(p, c)];
        else sv = fabs(F[c]);
        s += wb[j] * sv;
      }
      sc[g] = s;
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* surface quantities (Sec. 6)                                               */
/* ------------------------------------------------------------------------- */

/* Field values on the 2^d points G, P1.. of ghost g's stencil box (all
 * corners; a corner outside the grid reads as NaN). */
static void box_values(const orc_plan* p, int64_t g, const double* F, double* v) {
  int dim = p->dim;
  int64_t ijk[3];
  unlinear(&p->g, p->cell[g], ijk);
  v[0] = F[p->cell[g]];
  for (int k = 0; k < npts(dim); ++k) {
    const int* sb = subset(dim, k);
    int64_t q[3] = {ijk[0], ijk[1], ijk[2]};
    int ok = 1;
    for (int i = 0; i < dim; ++i)
      if (sb[i]) {
        q[i] += (int64_t)p->e[i * p->ng + g] * p->r[i * p->ng + g];
        if (q[i] < 0 || q[i] >= p->g.n[i]) ok = 0;
      }
    v[k + 1] = ok ? F[linear(&p->g, q)] : NAN;
  }
}

/* Value and gradient of the reconstruction polynomial of ghost g at the
 * point whose coordinates relative to G are xs.  Value: the bilinear /
 * trilinear interpolant through the stencil box; gradient: Eq.
 * derivative_bilinear (2D) and Eqs. derivative_trilinear_x/y/z (3D). */
static void eval_poly(const orc_plan* p, int64_t g, const double* pv,
                      const double xs_in[3], double* val, double* grad) {
  double x2[3], xs0[3], n[3];
  local_coords(p, g, x2, xs0, n);
  const double x1 = 0.0, y1 = 0.0, z1 = 0.0;
  double X2 = x2[0], Y2 = x2[1], Z2 = x2[2];
  double xs = xs_in[0], ys = xs_in[1], zs = xs_in[2];
  if (p->dim == 2) {
    double pG = pv[0], p1 = pv[1], p2 = pv[2], p3 = pv[3];
    double ax = (xs - x1) / (X2 - x1), ay = (ys - y1) / (Y2 - y1);
    *val = (1 - ax) * (1 - ay) * pG + ax * (1 - ay) * p1 + (1 - ax) * ay * p2 +
           ax * ay * p3;
    grad[0] = ((Y2 - ys) / (Y2 - y1)) * ((p1 - pG) / (X2 - x1)) +
              ((ys - y1) / (Y2 - y1)) * ((p3 - p2) / (X2 - x1));
    grad[1] = ((X2 - xs) / (X2 - x1)) * ((p2 - pG) / (Y2 - y1)) +
              ((xs - x1) / (X2 - x1)) * ((p3 - p1) / (Y2 - y1));
  } else {
    double pG = pv[0], p1 = pv[1], p2 = pv[2], p3 = pv[3], p4 = pv[4],
           p5 = pv[5], p6 = pv[6], p7 = pv[7];
    double ax = (xs - x1) / (X2 - x1), ay = (ys - y1) / (Y2 - y1),
           az = (zs - z1) / (Z2 - z1);
    *val = (1 - ax) * (1 - ay) * (1 - az) * pG + ax * (1 - ay) * (1 - az) * p1 +
           (1 - ax) * ay * (1 - az) * p2 + (1 - ax) * (1 - ay) * az * p3 +
           ax * ay * (1 - az) * p4 + (1 - ax) * ay * az * p5 +
           ax * (1 - ay) * az * p6 + ax * ay * az * p7;
    double Ym = (Y2 - ys) / (Y2 - y1), Yp = (ys - y1) / (Y2 - y1);
    double Zm = (Z2 - zs) / (Z2 - z1), Zp = (zs - z1) / (Z2 - z1);
    double Xm = (X2 - xs) / (X2 - x1), Xp = (xs - x1) / (X2 - x1);
    grad[0] = Ym * Zm * ((p1 - pG) / (X2 - x1)) + Yp * Zm * ((p4 - p2) / (X2 - x1)) +
              Ym * Zp * ((p6 - p3) / (X2 - x1)) + Yp * Zp * ((p7 - p5) / (X2 - x1));
    grad[1] = Xm * Zm * ((p2 - pG) / (Y2 - y1)) + Xp * Zm * ((p4 - p1) / (Y2 - y1)) +
              Xm * Zp * ((p5 - p3) / (Y2 - y1)) + Xp * Zp * ((p7 - p6) / (Y2 - y1));
    grad[2] = Xm * Ym * ((p3 - pG) / (Z2 - z1)) + Xp * Ym * ((p6 - p1) / (Z2 - z1)) +
              Xm * Yp * ((p5 - p2) / (Z2 - z1)) + Xp * Yp * ((p7 - p4) / (Z2 - z1));
  }
}

int orc_surface_ghost(const orc_plan* p, int nf, const double* fields,
                      double* val, double* grad) {
  int64_t ng = p->ng;
  int dim = p->dim;
  for (int f = 0; f < nf; ++f) {
    const double* F = fields + (int64_t)f * p->ncell;
    for (int64_t g = 0; g < ng; ++g) {
      double pv[8], xs[3] = {0, 0, 0}, v, gr[3];
      box_values(p, g, F, pv);
      for (int i = 0; i < dim; ++i) xs[i] = p->delta[i * ng + g];
      eval_poly(p, g, pv, xs, &v, gr);
      val[(int64_t)f * ng + g] = v;
      for (int i = 0; i < dim; ++i) grad[((int64_t)f * dim + i) * ng + g] = gr[i];
    }
  }
  return ORC_OK;
}

/* Anchor ghost of a query point: the ghost, among those whose cell lies
 * within 2 cells per axis of the cell containing x, with the smallest
 * |x - S_G|^2; ties go to the smaller linear index. */
static int64_t find_anchor(const orc_plan* p, const double* x) {
  int dim = p->dim;
  int64_t qi[3] = {0, 0, 0};
  for (int i = 0; i < dim; ++i) qi[i] = cell_of(&p->g, i, x[i]);
  int64_t best = -1;
  double bd = INFINITY;
  int64_t kz0 = dim == 3 ? qi[2] - 2 : 0, kz1 = dim == 3 ? qi[2] + 2 : 0;
  for (int64_t k = kz0; k <= kz1; ++k)
    for (int64_t j = qi[1] - 2; j <= qi[1] + 2; ++j)
      for (int64_t i = qi[0] - 2; i <= qi[0] + 2; ++i) {
        int64_t q[3] = {i, j, k};
        int ok = 1;
        for (int a = 0; a < dim; ++a) if (q[a] < 0 || q[a] >= p->g.n[a]) ok = 0;
        if (!ok) continue;
        int64_t c = linear(&p->g, q);
        if (p->tag[c] != 2 && p->tag[c] != -2) continue;
        int64_t g = find_ghost(p, c);
        double d2 = 0.0;
        for (int a = 0; a < dim; ++a) {
          double s = centre(&p->g, a, q[a]) + p->delta[a * p->ng + g];
          d2 += (x[a] - s) * (x[a] - s);
        }
        if (d2 < bd) { bd = d2; best = g; }
      }
  return best;
}

int orc_surface_query(const orc_plan* p, int64_t nq, const double* xq, int nf,
                      const double* fields, double* val, double* grad,
                      int64_t* anchor, const double* field_scale, double* scale) {
  int dim = p->dim;
  for (int64_t q = 0; q < nq; ++q) {
    double x[3] = {0, 0, 0};
    for (int i = 0; i < dim; ++i) x[i] = xq[i * nq + q];
    int64_t g = find_anchor(p, x);
    if (g < 0) return ORC_E_STENCIL;
    if (anchor) anchor[q] = g;
    int64_t ijk[3];
    unlinear(&p->g, p->cell[g], ijk);
    double rel[3] = {0, 0, 0};
    for (int i = 0; i < dim; ++i) rel[i] = x[i] - centre(&p->g, i, ijk[i]);
    for (int f = 0; f < nf; ++f) {
      const double* F = fields + (int64_t)f * p->ncell;
      double pv[8], v, gr[3];
      box_values(p, g, F, pv);
      eval_poly(p, g, pv, rel, &v, gr);
      if (val) val[(int64_t)f * nq + q] = v;
      if (grad)
        for (int i = 0; i < dim; ++i) grad[((int64_t)f * dim + i) * nq + q] = gr[i];
      if (scale && field_scale) {
        /* |coefficients| against the corner scales */
        const double* FS = field_scale + (int64_t)f * p->ncell;
        double sv[8];
        box_values(p, g, FS, sv);
        int nc = 1 << dim;
        double acc[4] = {0, 0, 0, 0};
        for (int c = 0; c < nc; ++c) {
          double unit[8] = {0, 0, 0, 0, 0, 0, 0, 0}, uv, ug[3];
          unit[c] = 1.0;
          eval_poly(p, g, unit, rel, &uv, ug);
          acc[0] += fabs(uv) * sv[c];
          for (int i = 0; i < dim; ++i) acc[1 + i] += fabs(ug[i]) * sv[c];
        }
        for (int i = 0; i <= dim; ++i) scale[((int64_t)f * (dim + 1) + i) * nq + q] = acc[i];
      }
    }
  }
  return ORC_OK;
}

int orc_forces(const orc_plan* p, int64_t nq, const double* xq,
               const double* nrm, const double* wq, const double* pfield,
               const double* u, double mu, double* F) {
  /* traction -p n + mu (grad u + grad u^T) n, summed with weights w_q */
  int dim = p->dim;
  double* pv = (double*)malloc(sizeof(double) * (nq ? nq : 1));
  double* ug = (double*)malloc(sizeof(double) * dim * dim * (nq ? nq : 1));
  int st = orc_surface_query(p, nq, xq, 1, pfield, pv, NULL, NULL, NULL, NULL);
  if (st == ORC_OK)
    st = orc_surface_query(p, nq, xq, dim, u, NULL, ug, NULL, NULL, NULL);
  for (int i = 0; i < dim; ++i) F[i] = 0.0;
  if (st == ORC_OK) {
    for (int64_t q = 0; q < nq; ++q) {
      for (int i = 0; i < dim; ++i) {
        double t = -pv[q] * nrm[i * nq + q];
        for (int j = 0; j < dim; ++j) {
          /* d u_i / d x_j = ug[(i*dim + j)*nq + q] */
          double dij = ug[((int64_t)i * dim + j) * nq + q];
          double dji = ug[((int64_t)j * dim + i) * nq + q];
          t += mu * (dij + dji) * nrm[j * nq + q];
        }
        F[i] += wq[q] * t;
      }
    }
  }
  free(pv); free(ug);
  return st;
}

/* ------------------------------------------------------------------------- */
/* adjoints: explicit transposes of the linear maps above                    */
/* ------------------------------------------------------------------------- */

/* lam[c] += sum_q (L_c(x_q) gval_q + grad L_c(x_q) . ggrad_q) over the
 * corners c of each query's anchor box; with absval, the magnitude of every
 * term is added instead (the scale of the sum). */
static int surface_adjoint(const orc_plan* p, int64_t nq, const double* xq,
                           int nf, const double* gval, const double* ggrad,
                           double* lam, int absval) {
  int dim = p->dim, nc = 1 << dim;
  for (int64_t q = 0; q < nq; ++q) {
    double x[3] = {0, 0, 0};
    for (int i = 0; i < dim; ++i) x[i] = xq[i * nq + q];
    int64_t g = find_anchor(p, x);
    if (g < 0) return ORC_E_STENCIL;
    int64_t ijk[3];
    unlinear(&p->g, p->cell[g], ijk);
    double rel[3] = {0, 0, 0};
    for (int i = 0; i < dim; ++i) rel[i] = x[i] - centre(&p->g, i, ijk[i]);
    /* corner cells in the box_values order */
    int64_t cc[8];
    cc[0] = p->cell[g];
    for (int k = 0; k < npts(dim); ++k) {
      const int* sb = subset(dim, k);
      int64_t qq[3] = {ijk[0], ijk[1], ijk[2]};
      for (int i = 0; i < dim; ++i)
        if (sb[i]) qq[i] += (int64_t)p->e[i * p->ng + g] * p->r[i * p->ng + g];
      cc[k + 1] = linear(&p->g, qq);
    }
    for (int c = 0; c < nc; ++c) {
      double unit[8] = {0, 0, 0, 0, 0, 0, 0, 0}, uv, ug[3];
      unit[c] = 1.0;
      eval_poly(p, g, unit, rel, &uv, ug);
      for (int f = 0; f < nf; ++f) {
        double a;
        if (!absval) {
          a = gval ? uv * gval[(int64_t)f * nq + q] : 0.0;
          if (ggrad)
            for (int i = 0; i < dim; ++i) a += ug[i] * ggrad[((int64_t)f * dim + i) * nq + q];
        } else {
          a = gval ? fabs(uv * gval[(int64_t)f * nq + q]) : 0.0;
          if (ggrad)
            for (int i = 0; i < dim; ++i)
              a += fabs(ug[i] * ggrad[((int64_t)f * dim + i) * nq + q]);
        }
        lam[(int64_t)f * p->ncell + cc[c]] += a;
      }
    }
  }
  return ORC_OK;
}

int orc_surface_query_adjoint(const orc_plan* p, int64_t nq, const double* xq,
                              int nf, const double* gval, const double* ggrad,
                              double* lam) {
  return surface_adjoint(p, nq, xq, nf, gval, ggrad, lam, 0);
}

int orc_surface_query_adjoint_scale(const orc_plan* p, int64_t nq,
                                    const double* xq, int nf,
                                    const double* gval, const double* ggrad,
                                    double* lam_scale) {
  return surface_adjoint(p, nq, xq, nf, gval, ggrad, lam_scale, 1);
}

int orc_fill_adjoint(const orc_plan* p, int nf, double* lam,
                     const int8_t* bc_type, double* lam_bc) {
  /* reverse canonical order: Lambda_G = lam[G]; lam_bc = w_s Lambda_G;
   * lam[P_k] += w_k Lambda_G; the ghost's own input slot is overwritten by
   * the fill, so its sensitivity is zero.  A coupled unit solves the
   * transposed system A^T mu = Lambda first. */
  int64_t ng = p->ng;
  for (int f = 0; f < nf; ++f) {
    double* L = lam + (int64_t)f * p->ncell;
    const int8_t* bt = bc_type + (int64_t)f * ng;
    double* lb = lam_bc + (int64_t)f * ng;
    for (int64_t g = ng - 1; g >= 0; --g) {
      int32_t u = p->blk[g];
      if (u < 0) {
        double w[7], ws;
        orc_weights(p, g, bt[g], w, &ws);
        double Lg = L[p->cell[g]];
        lb[g] = ws * Lg;
        L[p->cell[g]] = 0.0;
        for (int j = 0; j < npts(p->dim); ++j) {
          int64_t c = p->sten[7 * g + j];
          if (c >= 0) L[c] += w[j] * Lg;
        }
        continue;
      }
      if (g != p->blk_mem[p->blk_off[u + 1] - 1]) continue;
      const int32_t k = unit_size(p, u);
      const int64_t* m = p->blk_mem + p->blk_off[u];
      double* A = (double*)malloc(sizeof(double) * (2 * k * k + 2 * k));
      if (!A) return ORC_E_NOMEM;
      double* AT = A + (int64_t)k * k;
      double* mu = AT + (int64_t)k * k;
      double* dummy = mu + k;
      unit_system(p, u, NULL, bt, NULL, A, dummy, 0, NULL);   /* matrix only */
      for (int i = 0; i < k; ++i)
        for (int t = 0; t < k; ++t) AT[i * k + t] = A[t * k + i];
      for (int i = 0; i < k; ++i) mu[i] = L[p->cell[m[i]]];
      int st = gauss(k, AT, mu);
      if (st != ORC_OK) { free(A); return st; }
      for (int i = 0; i < k; ++i) L[p->cell[m[i]]] = 0.0;
      for (int i = 0; i < k; ++i) {
        double w[7], ws;
        orc_weights(p, m[i], bt[m[i]], w, &ws);
        lb[m[i]] = ws * mu[i];
        for (int j = 0; j < npts(p->dim); ++j) {
          int64_t c = p->sten[7 * m[i] + j];
          if (c < 0) continue;
          int internal = 0;
          for (int q = 0; q < k; ++q) if (p->cell[m[q]] == c) internal = 1;
          if (!internal) L[c] += w[j] * mu[i];
        }
      }
      free(A);
    }
  }
  return ORC_OK;
}

int orc_fill_adjoint_scale(const orc_plan* p, int nf, double* lam_scale,
                           const int8_t* bc_type, double* lam_bc_scale) {
  /* The reverse sweep of orc_fill_adjoint with every weight replaced by its
   * bound (orc_weight_bounds) and the unit solves by |A^-T|: each output
   * receives the sum of the magnitudes of the terms that make it up, the
   * scale of its error.  Ghost slots end at zero, as the adjoint's do. */
  int64_t ng = p->ng;
  for (int f = 0; f < nf; ++f) {
    double* L = lam_scale + (int64_t)f * p->ncell;
    const int8_t* bt = bc_type + (int64_t)f * ng;
    double* lb = lam_bc_scale + (int64_t)f * ng;
    for (int64_t g = ng - 1; g >= 0; --g) {
      int32_t u = p->blk[g];
      if (u < 0) {
        double wb[7], wsb;
        orc_weight_bounds(p, g, bt[g], wb, &wsb);
        double Lg = L[p->cell[g]];
        lb[g] = wsb * Lg;
        L[p->cell[g]] = 0.0;
        for (int j = 0; j < npts(p->dim); ++j) {
          int64_t c = p->sten[7 * g + j];
          if (c >= 0) L[c] += wb[j] * Lg;
        }
        continue;
      }
      if (g != p->blk_mem[p->blk_off[u + 1] - 1]) continue;
      const int32_t k = unit_size(p, u);
      const int64_t* m = p->blk_mem + p->blk_off[u];
      double* inv = unit_abs_inverse(p, u, bt);
      double* mu = (double*)malloc(sizeof(double) * k);
      if (!inv || !mu) { free(inv); free(mu); return ORC_E_NOMEM; }
      /* |A^-T| s: entry i sums |(A^-1)_{t i}| s_t */
      for (int i = 0; i < k; ++i) {
        double acc = 0.0;
        for (int t = 0; t < k; ++t) acc += inv[t * k + i] * L[p->cell[m[t]]];
        mu[i] = acc;
      }
      for (int i = 0; i < k; ++i) L[p->cell[m[i]]] = 0.0;
      for (int i = 0; i < k; ++i) {
        double wb[7], wsb;
        orc_weight_bounds(p, m[i], bt[m[i]], wb, &wsb);
        lb[m[i]] = wsb * mu[i];
        for (int j = 0; j < npts(p->dim); ++j) {
          int64_t c = p->sten[7 * m[i] + j];
          if (c < 0) continue;
          int internal = 0;
          for (int q = 0; q < k; ++q) if (p->cell[m[q]] == c) internal = 1;
          if (!internal) L[c] += wb[j] * mu[i];
        }
      }
      free(inv); free(mu);
    }
  }
  return ORC_OK;
}
