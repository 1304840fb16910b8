/*
 * oracle.h -- CPU reference ("oracle") for the direct, non-iterative ghost-cell
 * method of Rapaka, Jagad, Addad & Riahi, "Stable, Compact, and Direct
 * Ghost-Cell Reconstruction".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU baseline
 * leg of the benchmark do.  It shares no code with the GPU path.
 *
 * Plain C99, FP64, scalar loops, built with -ffp-contract=off.  All arrays are
 * host memory owned by the caller unless stated otherwise.  Cell (i,j,k) of a
 * grid has centre lo + (idx + 1/2) h per axis and linear index
 * i + n0 (j + n1 k) (x fastest).
 */
#ifndef GCR_ORACLE_H
#define GCR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0, ORC_E_ARG = 1, ORC_E_NOMEM = 3, ORC_E_CYCLE = 4,
  ORC_E_STENCIL = 5, ORC_E_DEGENERATE = 6, ORC_E_GEOMETRY = 7,
  ORC_E_UNSUPPORTED = 8
};
enum { ORC_SPHERE = 0, ORC_STAR2D = 1, ORC_SHSTAR = 2, ORC_AIRFOIL = 3 };
enum { ORC_CGC = 0, ORC_CGC_ES = 1, ORC_HGC = 2 };
/* Flag added to a scheme: a second ghost layer (Sec. 7.1), solid cells with
 * psi <= 1.5 delta n, on the extended stencil of Eq. stencil_anisotropic. */
enum { ORC_LAYER2 = 4 };
enum { ORC_DIRICHLET = 0, ORC_NEUMANN = 1 };

/* Uniform spacing h per axis from lo, or, where faces[i] is given, the n[i]
 * + 1 cell faces of axis i (strictly increasing; lo and h then unused on
 * that axis): a stretched grid, with cell centres midway between faces and
 * the local spacing of a cell its width. */
typedef struct {
  int32_t dim, pad;
  int64_t n[3];
  double lo[3];
  double h[3];
  const double* faces[3];
} orc_grid;

/*
 * kind ORC_SPHERE : circle (2D) / sphere (3D) of radius r0 about c.
 * kind ORC_STAR2D : r(theta) = r0 (1 + sum_k A_k cos k theta + B_k sin k theta),
 *                   coef = {A_0,B_0, A_1,B_1, ...}, ncoef = number of k values.
 * kind ORC_SHSTAR : r(omega) = r0 (1 + sum_{l,m} a_lm Y_lm(omega)), real
 *                   Schmidt semi-normalised harmonics without Condon-Shortley
 *                   phase, coef[l*l + l + m], ncoef = (L+1)^2.
 * kind ORC_AIRFOIL: symmetric four-digit thickness form, chord `chord`,
 *                   thickness ratio `thick`, leading edge at c, pitched nose-up
 *                   by `incidence` radians, closed trailing edge.
 */
typedef struct {
  int32_t kind, ncoef;
  double c[3];
  double r0;
  const double* coef;
  double chord, thick, incidence;
} orc_shape;

typedef struct orc_plan orc_plan;

int orc_plan_create(const orc_grid* g, const orc_shape* s, int scheme,
                    orc_plan** out);
void orc_plan_destroy(orc_plan* p);
int64_t orc_n_cells(const orc_plan* p);
int64_t orc_n_ghost(const orc_plan* p);
int64_t orc_n_interface(const orc_plan* p);
int32_t orc_n_levels(const orc_plan* p);
int orc_dim(const orc_plan* p);

/* Level-sorted (canonical: level ascending, linear index ascending) export.
 * Any pointer may be NULL.  delta/normal/r are [dim][N_g]. */
void orc_export(const orc_plan* p, int8_t* tags, int64_t* ghost_cell,
                int32_t* level_off, int32_t* level, double* delta,
                double* normal, double* psi, int32_t* r);
/* Stencil cells of ghost g (canonical position): [2^d - 1], -1 where skipped. */
void orc_stencil(const orc_plan* p, int64_t g, int64_t* cells);
/* Decision margins (in units of h): [0] classification, [1] HGC band and
 * second-layer threshold,
 * [2] CGC_ES multiplier, [3] normal sign, [4] max alpha_x, [5] max alpha_y,
 * [6] max alpha_z. */
void orc_margins(const orc_plan* p, double* out);
/* Coupled units (strongly connected components of the ghost graph with more
 * than one ghost): count, largest size, and per ghost (canonical order) the
 * unit id or -1. */
void orc_units(const orc_plan* p, int32_t* nblk, int32_t* maxblk, int32_t* unit);
/* Reconstruction weights of ghost g: w[2^d-1] on P1..P(2^d-1) (paper order)
 * and ws on the boundary datum. */
int orc_weights(const orc_plan* p, int64_t g, int bc, double* w, double* ws);
/* Same from raw local geometry: x2 = r e dx, xs = x_s - x_1, n (all [dim]). */
int orc_weights_raw(int dim, int bc, const double* x2, const double* xs,
                    const double* n, double* w, double* ws);
/* Tolerance bounds of the same weights: wb[k] = |w_k| + sum_i (|x2_i|
 * |dw_k/dxs_i| + |dw_k/dn_i|), wsb likewise for w_s: their magnitude plus
 * how far they move when the foot point moves on the scale of the stencil
 * span and the normal on the scale of a unit vector (each side of a parity
 * comparison projects the body on its own). */
int orc_weight_bounds_raw(int dim, int bc, const double* x2, const double* xs,
                          const double* n, double* wb, double* wsb);
int orc_weight_bounds(const orc_plan* p, int64_t g, int bc, double* wb, double* wsb);

/* Fresh cells of a moved body (Sec. 7.1: moving boundaries expose fresh
 * fluid cells, one reason for a second ghost layer).  a: the plan before the
 * move, b: after, on the same grid.  A cell is fresh when its centre was
 * solid in a (tag 1 or 2) and is fluid in b (tag 0 or -2); it is uncovered
 * when it was not a ghost of a (tag 1: its value was never reconstructed).
 * list (may be NULL) receives the fresh cells' linear indices, ascending,
 * up to cap of them; the counts are always complete.  Returns ORC_E_ARG if
 * the grids differ. */
int orc_fresh_cells(const orc_plan* a, const orc_plan* b, int64_t* n_fresh,
                    int64_t* n_uncovered, int64_t* list, int64_t cap);

/* Fill.  fields: [nf][N_cells] in/out.  bc_type: [nf][N_g] (0 Dirichlet,
 * 1 Neumann).  bc_val: [nf][N_g] values at S (phi_s or dphi/dn). */
int orc_fill(const orc_plan* p, int nf, double* fields, const int8_t* bc_type,
             const double* bc_val);
/* Synchronous (Jacobi) sweeps of the same relations, from NaN ghosts, until
 * a fixed point; returns the number of sweeps after which every ghost was
 * final (or -1 if max_sweeps reached). */
int orc_fill_jacobi(const orc_plan* p, int nf, double* fields,
                    const int8_t* bc_type, const double* bc_val,
                    int max_sweeps);
/* Condition-aware scale of every filled ghost value: [nf][N_g].  s_G sums
 * wb_k s_{P_k} over the stencil (s = |phi| on non-ghost cells) and
 * wsb |b_G|, with the weight bounds above; a coupled unit takes |A^-1|
 * times its external sums. */
int orc_fill_scale(const orc_plan* p, int nf, const double* fields,
                   const int8_t* bc_type, const double* bc_val, double* scale);

/* Boundary value and Cartesian gradient at every ghost's foot point S.
 * val [nf][N_g], grad [nf][dim][N_g]. */
int orc_surface_ghost(const orc_plan* p, int nf, const double* fields,
                      double* val, double* grad);
/* Same at query points xq [dim][nq] via the anchor ghost (closest S among
 * ghosts within 2 cells per axis of the query's cell).  anchor [nq] gets the
 * canonical position of the anchor.  scale (optional) [nf][(1+dim)][nq]. */
int orc_surface_query(const orc_plan* p, int64_t nq, const double* xq, int nf,
                      const double* fields, double* val, double* grad,
                      int64_t* anchor, const double* field_scale,
                      double* scale);
/* Pressure + viscous force F[dim] = sum_q w_q (-p n + mu (grad u + grad u^T) n).
 * u: [dim][N_cells]. */
int orc_forces(const orc_plan* p, int64_t nq, const double* xq,
               const double* nrm, const double* wq, const double* pfield,
               const double* u, double mu, double* F);

/* Adjoints.  lam: [nf][N_cells] dense; surface adjoint adds into it. */
int orc_surface_query_adjoint(const orc_plan* p, int64_t nq, const double* xq,
                              int nf, const double* gval, const double* ggrad,
                              double* lam);
/* lam in: dJ/d(filled field); out: dJ/d(input field) (ghost slots zeroed).
 * lam_bc out: [nf][N_g].  Coupled units of any size are solved densely. */
int orc_fill_adjoint(const orc_plan* p, int nf, double* lam,
                     const int8_t* bc_type, double* lam_bc);

/* Condition-aware scales of the adjoints, for tolerances: the same sweeps
 * with every coefficient replaced by its magnitude (a relation's weights by
 * their bounds, a unit's solve by |A^-T|), so each output receives the sum
 * of the magnitudes of the terms that make it up.  surface: adds into lam_scale [nf][N_cells] from the
 * magnitudes of gval, ggrad; fill: lam_scale in = scale of dJ/d(filled),
 * out = scale of dJ/d(input) (ghost slots zero); lam_bc_scale [nf][N_g]. */
int orc_surface_query_adjoint_scale(const orc_plan* p, int64_t nq,
                                    const double* xq, int nf,
                                    const double* gval, const double* ggrad,
                                    double* lam_scale);
int orc_fill_adjoint_scale(const orc_plan* p, int nf, double* lam_scale,
                           const int8_t* bc_type, double* lam_bc_scale);

/* Geometry helpers exposed for pins. */
int orc_shape_project(const orc_shape* s, int dim, const double* x, int solid,
                      double* S, double* n, double* psi);
int orc_shape_inside(const orc_shape* s, int dim, const double* x);
double orc_shape_radius(const orc_shape* s, int dim, const double* omega);
double orc_sh_basis(int l, int m, const double* v);

#ifdef __cplusplus
}
#endif
#endif
