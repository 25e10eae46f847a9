/*
 * lr_ref.c — FP64 CPU oracle of one DirectCF Lagrange–Remap time step.
 *
 * TEST INFRASTRUCTURE ONLY (see lr_ref.h).  Nothing in the GPU library links,
 * includes or calls this file.
 *
 * The step follows the paper in its own order:
 *   §1.2  SGPC predictor (eq. "prediction") and corrector (eq. "correction"),
 *         the quad-cell volume F, the nodal pressure gradient, nodal mass and
 *         the discrete Wilkins pseudo-viscosity;
 *   §4.1  the iso-deformation multimaterial form of both phases
 *         (eqs. "prediction_multi", "correction_multi"), mixed-cell pressure,
 *         Youngs normals;
 *   §2.3  DirectCF corner and face volume fluxes, the flux-consistent
 *         Lagrangian volume, the primal and dual (momentum) remap;
 *   §2.1.1 / §3.3  upwind, limited linear (Van Leer) face reconstruction and
 *         the linear diagonal corner reconstruction;
 *   §4.4  interface placed on the rectangular approximation of the Lagrangian
 *         cell and partial volume fluxes from its intersection with every
 *         face and corner flux volume;
 *   §5.1, §5.2  perfect-gas and stiffened-gas equations of state.
 * The alternate-direction remap of §2.1.1-§2.1.2 and §4.2, the paper's
 * comparator, replaces the DirectCF remap when opts.remap asks for it.
 * Where the paper is silent the readings are the ones written in the design
 * notes of this repository (donor-side volume-fraction clipping, mixture sound
 * speed, CFL formula, boundary mirrors, dual-mesh geometry, ...); each such
 * place is marked "reading".
 *
 * Style: whole-array stages with explicit ghost layers filled by mirroring,
 * polygon clipping for every intersection and bisection for the interface
 * offset — slow on purpose, so that each stage can be checked by eye.
 */
#include "lr_ref.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define G 2 /* ghost layers on every array */

/* branch flags of a cell in one step; counted per step in ctx->counts */
enum {
  F_MIXED = 1,      /* two or more materials present: interface reconstructed */
  F_THREE = 2,      /* three or more materials present                          */
  F_DEGENERATE = 4, /* a Youngs gradient too small to give a normal             */
  F_CLIPPED = 8,    /* donor-side limiting of a material's outflow applied      */
  F_GUARD = 16      /* positivity guard: the donor fell back to order 1         */
};

struct lr_ref_ctx {
  int nx, ny, nmat;
  lr_ref_eos eos[LR_REF_MAXMAT];
  lr_ref_opts o;
  double dx, dy, A;
  double t;
  long step;
  int have_state;
  char err[256];
  /* padded sizes */
  int cw, ch;     /* cells:   (nx+2G) x (ny+2G)     */
  int nw, nh;     /* nodes:   (nx+1+2G) x (ny+1+2G) */
  /* persistent state */
  double *V, *M, *E;   /* [nmat][cells] partial volume, mass, internal energy */
  double *ux, *uy;     /* [nodes] */
  /* stage arrays kept from the last step (debug / pins) */
  double *k, *rho_a, *e_a, *P_a, *Pc, *cc, *rhoc, *Mc, *Q;
  double *e_half, *P_half, *Pc_half, *S;
  double *mp, *uhx, *uhy, *uLx, *uLy, *dpx, *dpy, *xLx, *xLy;
  double *VL, *eL;
  double *volcf, *rhocf, *xcL, *ycL, *dxL, *dyL;
  int *pure; /* material index if exactly one material present, -1 if mixed */
  int *flags; /* branches a cell took in the last step (F_* bits below) */
  long counts[LR_REF_NCOUNT]; /* cells that took each branch, summed since set_state */
  double *muX, *muY, *muD, *muA; /* signed total mass fluxes (padded) */
  double *Wx, *Wy, *Wc;          /* signed face / corner volume fluxes (real) */
  double *Wpx, *Wpy, *Wpc;       /* per-material partial volumes [nmat][...] */
  double last_dt;
};

/* ------------------------------------------------------------------------ */
/* indexing                                                                  */
static inline int CI(const lr_ref_ctx *c, int i, int j) { return (j + G) * c->cw + (i + G); }
static inline int NI(const lr_ref_ctx *c, int I, int J) { return (J + G) * c->nw + (I + G); }
/* x-faces share the node column index and the cell row index */
static inline int XI(const lr_ref_ctx *c, int I, int j) { return (j + G) * c->nw + (I + G); }
/* y-faces share the cell column index and the node row index */
static inline int YI(const lr_ref_ctx *c, int i, int J) { return (J + G) * c->cw + (i + G); }
static inline int ncell(const lr_ref_ctx *c) { return c->cw * c->ch; }
static inline int nnode(const lr_ref_ctx *c) { return c->nw * c->nh; }
static inline int nxf(const lr_ref_ctx *c) { return c->nw * c->ch; }
static inline int nyf(const lr_ref_ctx *c) { return c->cw * c->nh; }

/* mirror of a cell index about the walls (reflective boundary, reading) */
static int mc(int i, int n) { return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i); }
/* mirror of a node index about the walls */
static int mn(int I, int n) { return I < 0 ? -I : (I > n ? 2 * n - I : I); }

static double node_x(const lr_ref_ctx *c, int I) { return c->o.x0 + I * c->dx; }
static double node_y(const lr_ref_ctx *c, int J) { return c->o.y0 + J * c->dy; }

static int fail(lr_ref_ctx *c, int code, const char *msg) {
  snprintf(c->err, sizeof c->err, "%s", msg);
  return code;
}

/* ghost cells copy the mirrored real cell (scalars) */
static void ghost_cells(const lr_ref_ctx *c, double *a) {
  for (int j = -G; j < c->ny + G; ++j)
    for (int i = -G; i < c->nx + G; ++i) {
      int ri = mc(i, c->nx), rj = mc(j, c->ny);
      if (ri != i || rj != j) a[CI(c, i, j)] = a[CI(c, ri, rj)];
    }
}
static void ghost_cells_int(const lr_ref_ctx *c, int *a) {
  for (int j = -G; j < c->ny + G; ++j)
    for (int i = -G; i < c->nx + G; ++i) {
      int ri = mc(i, c->nx), rj = mc(j, c->ny);
      if (ri != i || rj != j) a[CI(c, i, j)] = a[CI(c, ri, rj)];
    }
}
/* ghost cells of a cell-centre x (or y) coordinate: reflected position */
static void ghost_cells_coord(const lr_ref_ctx *c, double *a, int axis) {
  for (int j = -G; j < c->ny + G; ++j)
    for (int i = -G; i < c->nx + G; ++i) {
      int ri = mc(i, c->nx), rj = mc(j, c->ny);
      if (ri == i && rj == j) continue;
      double v = a[CI(c, ri, rj)];
      if (axis == 0 && ri != i) v = 2.0 * (i < 0 ? c->o.x0 : c->o.x1) - v;
      if (axis == 1 && rj != j) v = 2.0 * (j < 0 ? c->o.y0 : c->o.y1) - v;
      a[CI(c, i, j)] = v;
    }
}
/* ghost nodes of a nodal vector (vx, vy): the normal component flips sign */
static void ghost_nodes_vec(const lr_ref_ctx *c, double *vx, double *vy) {
  for (int J = -G; J <= c->ny + G; ++J)
    for (int I = -G; I <= c->nx + G; ++I) {
      int rI = mn(I, c->nx), rJ = mn(J, c->ny);
      if (rI == I && rJ == J) continue;
      double ax = vx[NI(c, rI, rJ)], ay = vy[NI(c, rI, rJ)];
      if (rI != I) ax = -ax;
      if (rJ != J) ay = -ay;
      vx[NI(c, I, J)] = ax;
      vy[NI(c, I, J)] = ay;
    }
}
/* ghost nodes of nodal positions: reflected about the wall */
static void ghost_nodes_pos(const lr_ref_ctx *c, double *px, double *py) {
  for (int J = -G; J <= c->ny + G; ++J)
    for (int I = -G; I <= c->nx + G; ++I) {
      int rI = mn(I, c->nx), rJ = mn(J, c->ny);
      if (rI == I && rJ == J) continue;
      double ax = px[NI(c, rI, rJ)], ay = py[NI(c, rI, rJ)];
      if (rI != I) ax = 2.0 * (I < 0 ? c->o.x0 : c->o.x1) - ax;
      if (rJ != J) ay = 2.0 * (J < 0 ? c->o.y0 : c->o.y1) - ay;
      px[NI(c, I, J)] = ax;
      py[NI(c, I, J)] = ay;
    }
}
static void ghost_nodes_scalar(const lr_ref_ctx *c, double *a) {
  for (int J = -G; J <= c->ny + G; ++J)
    for (int I = -G; I <= c->nx + G; ++I) {
      int rI = mn(I, c->nx), rJ = mn(J, c->ny);
      if (rI != I || rJ != J) a[NI(c, I, J)] = a[NI(c, rI, rJ)];
    }
}

/* ------------------------------------------------------------------------ */
/* geometry                                                                  */

/* §1.2: F = 1/2 |dx_{i-1/2,j} ^ dx_{i,j-1/2}| + 1/2 |dx_{i+1/2,j} ^ dx_{i,j+1/2}|
 * with the left, bottom, right and top edge vectors of the quadrilateral. */
static double quad_F(double blx, double bly, double brx, double bry,
                     double tlx, double tly, double trx, double try_) {
  double Lx = tlx - blx, Ly = tly - bly; /* left edge   */
  double Bx = brx - blx, By = bry - bly; /* bottom edge */
  double Rx = trx - brx, Ry = try_ - bry; /* right edge  */
  double Tx = trx - tlx, Ty = try_ - tly; /* top edge    */
  return 0.5 * fabs(Lx * By - Ly * Bx) + 0.5 * fabs(Rx * Ty - Ry * Tx);
}

/* area of the part of rectangle [x0,x1]x[y0,y1] where nx*x + ny*y >= s:
 * Sutherland–Hodgman clip of the 4-gon against the half-plane, then shoelace */
double lr_ref_rect_halfplane_area(double x0, double x1, double y0, double y1,
                                  double nx, double ny, double s) {
  double px[8], py[8], qx[8], qy[8];
  int n = 4, m = 0;
  if (!(x1 > x0) || !(y1 > y0)) return 0.0;
  px[0] = x0; py[0] = y0;
  px[1] = x1; py[1] = y0;
  px[2] = x1; py[2] = y1;
  px[3] = x0; py[3] = y1;
  for (int a = 0; a < n; ++a) {
    int b = (a + 1) % n;
    double fa = nx * px[a] + ny * py[a] - s;
    double fb = nx * px[b] + ny * py[b] - s;
    if (fa >= 0) { qx[m] = px[a]; qy[m] = py[a]; ++m; }
    if ((fa >= 0) != (fb >= 0)) {
      double t = fa / (fa - fb);
      qx[m] = px[a] + t * (px[b] - px[a]);
      qy[m] = py[a] + t * (py[b] - py[a]);
      ++m;
    }
  }
  double area = 0.0;
  for (int a = 0; a < m; ++a) {
    int b = (a + 1) % m;
    area += qx[a] * qy[b] - qx[b] * qy[a];
  }
  area = 0.5 * fabs(area);
  double full = (x1 - x0) * (y1 - y0);
  return area > full ? full : area;
}

/* §4.4: the offset s of the line n.x = s such that the part of the rectangle
 * on the side n.x >= s has area frac*|R|; monotone bisection */
double lr_ref_interface_offset(double x0, double x1, double y0, double y1,
                               double nx, double ny, double frac) {
  double c0 = nx * x0 + ny * y0, c1 = nx * x1 + ny * y0;
  double c2 = nx * x1 + ny * y1, c3 = nx * x0 + ny * y1;
  double lo = fmin(fmin(c0, c1), fmin(c2, c3)); /* whole rectangle on the side */
  double hi = fmax(fmax(c0, c1), fmax(c2, c3)); /* nothing on the side         */
  double target = frac * (x1 - x0) * (y1 - y0);
  double tol = 1e-17 * (hi - lo);
  for (int it = 0; it < 200 && hi - lo > tol; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (lr_ref_rect_halfplane_area(x0, x1, y0, y1, nx, ny, mid) > target) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* Van Leer limited slope from the two one-sided slopes (§2.1.1):
 * 1/2 (phi(r) d+ + phi(1/r) d-) with phi(r) = (r+|r|)/(1+r), r = d-/d+;
 * for r > 0 this is the harmonic mean 2 d- d+ / (d- + d+), else 0 (reading). */
static double van_leer(double dm, double dp) {
  if (dm * dp <= 0.0) return 0.0;
  double r = dm / dp;
  double phi_r = (r + fabs(r)) / (1.0 + r);
  double ri = 1.0 / r;
  double phi_ri = (ri + fabs(ri)) / (1.0 + ri);
  return 0.5 * (phi_r * dp + phi_ri * dm);
}

/* Equation of state of material a.  §5.1 perfect gas p = (gamma-1) rho e;
 * §5.2 stiffened gas p = (gamma-1) rho e - pi as the paper writes it (pi = 0
 * is the perfect gas).  The squared sound speed is (dp/drho) at constant
 * entropy, (gamma-1)(e + p/rho) = (gamma p + pi)/rho. */
static double eos_p(const lr_ref_ctx *c, int a, double rho, double e) {
  return (c->eos[a].gamma - 1.0) * rho * e - c->eos[a].pinf;
}
static double eos_k_rho_c2(const lr_ref_ctx *c, int a, double k, double P) {
  return k * c->eos[a].gamma * P + k * c->eos[a].pinf; /* k rho_a c_a^2 */
}

/* ------------------------------------------------------------------------ */
/* allocation                                                                */
static double *dalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

void lr_ref_default_opts(lr_ref_opts *o) {
  memset(o, 0, sizeof *o);
  o->x0 = 0; o->x1 = 1; o->y0 = 0; o->y1 = 1;
  o->cfl = 0.5; o->a1 = 0.5; o->a2 = 1.0;
  o->precision = 0; o->recon_order = 2; o->kinematic = 0;
  o->k_eps = 1e-10; o->fixed_dt = 0.0;
}

int lr_ref_create(int nx, int ny, int nmat, const lr_ref_eos *eos, const int bc[4],
                  const lr_ref_opts *opts, lr_ref_ctx **out) {
  if (!out) return LR_REF_EINVAL;
  *out = NULL;
  if (nx < 2 || ny < 2 || nmat < 1 || nmat > LR_REF_MAXMAT || !eos) return LR_REF_EINVAL;
  if (bc)
    for (int s = 0; s < 4; ++s)
      if (bc[s] != 0) return LR_REF_EINVAL;
  for (int a = 0; a < nmat; ++a)
    if (!(eos[a].gamma > 1.0) || !(eos[a].pinf >= 0.0) || !isfinite(eos[a].pinf))
      return LR_REF_EINVAL;
  lr_ref_ctx *c = (lr_ref_ctx *)calloc(1, sizeof *c);
  if (!c) return LR_REF_ENOMEM;
  c->nx = nx; c->ny = ny; c->nmat = nmat;
  memcpy(c->eos, eos, nmat * sizeof *eos);
  if (opts) c->o = *opts; else lr_ref_default_opts(&c->o);
  if (!(c->o.x1 > c->o.x0) || !(c->o.y1 > c->o.y0) || !(c->o.cfl > 0) ||
      c->o.recon_order < 1 || c->o.recon_order > 3 || !(c->o.k_eps >= 0) ||
      (c->o.remap != LR_REF_REMAP_DIRECTCF && c->o.remap != LR_REF_REMAP_AD) ||
      (c->o.remap == LR_REF_REMAP_AD && c->o.recon_order == 3) ||
      c->o.fixed_dt < 0) {
    free(c);
    return LR_REF_EINVAL;
  }
  c->dx = (c->o.x1 - c->o.x0) / nx;
  c->dy = (c->o.y1 - c->o.y0) / ny;
  c->A = c->dx * c->dy;
  c->cw = nx + 2 * G; c->ch = ny + 2 * G;
  c->nw = nx + 1 + 2 * G; c->nh = ny + 1 + 2 * G;
  size_t C = ncell(c), N = nnode(c), m = nmat;
  c->V = dalloc(m * C); c->M = dalloc(m * C); c->E = dalloc(m * C);
  c->ux = dalloc(N); c->uy = dalloc(N);
  c->k = dalloc(m * C); c->rho_a = dalloc(m * C); c->e_a = dalloc(m * C); c->P_a = dalloc(m * C);
  c->Pc = dalloc(C); c->cc = dalloc(C); c->rhoc = dalloc(C); c->Mc = dalloc(C); c->Q = dalloc(C);
  c->e_half = dalloc(m * C); c->P_half = dalloc(m * C); c->Pc_half = dalloc(C); c->S = dalloc(C);
  c->mp = dalloc(N); c->uhx = dalloc(N); c->uhy = dalloc(N); c->uLx = dalloc(N); c->uLy = dalloc(N);
  c->dpx = dalloc(N); c->dpy = dalloc(N); c->xLx = dalloc(N); c->xLy = dalloc(N);
  c->VL = dalloc(C); c->eL = dalloc(m * C);
  c->volcf = dalloc(C); c->rhocf = dalloc(m * C); c->xcL = dalloc(C); c->ycL = dalloc(C);
  c->dxL = dalloc(C); c->dyL = dalloc(C);
  c->pure = (int *)calloc(C, sizeof(int));
  c->flags = (int *)calloc(C, sizeof(int));
  c->muX = dalloc(nxf(c)); c->muY = dalloc(nyf(c)); c->muD = dalloc(N); c->muA = dalloc(N);
  c->Wx = dalloc(nxf(c)); c->Wy = dalloc(nyf(c)); c->Wc = dalloc(N);
  c->Wpx = dalloc(m * nxf(c)); c->Wpy = dalloc(m * nyf(c)); c->Wpc = dalloc(m * N);
  if (!c->V || !c->M || !c->E || !c->ux || !c->uy || !c->k || !c->rho_a || !c->e_a ||
      !c->P_a || !c->Pc || !c->cc || !c->rhoc || !c->Mc || !c->Q || !c->e_half ||
      !c->P_half || !c->Pc_half || !c->S || !c->mp || !c->uhx || !c->uhy || !c->uLx ||
      !c->uLy || !c->dpx || !c->dpy || !c->xLx || !c->xLy || !c->VL || !c->eL ||
      !c->volcf || !c->rhocf || !c->xcL || !c->ycL || !c->dxL || !c->dyL || !c->pure || !c->flags ||
      !c->muX || !c->muY || !c->muD || !c->muA || !c->Wx || !c->Wy || !c->Wc || !c->Wpx ||
      !c->Wpy || !c->Wpc) {
    lr_ref_destroy(c);
    return LR_REF_ENOMEM;
  }
  *out = c;
  return LR_REF_OK;
}

void lr_ref_destroy(lr_ref_ctx *c) {
  if (!c) return;
  double *arrs[] = {c->V, c->M, c->E, c->ux, c->uy, c->k, c->rho_a, c->e_a, c->P_a, c->Pc,
                    c->cc, c->rhoc, c->Mc, c->Q, c->e_half, c->P_half, c->Pc_half, c->S,
                    c->mp, c->uhx, c->uhy, c->uLx, c->uLy, c->dpx, c->dpy, c->xLx, c->xLy,
                    c->VL, c->eL, c->volcf, c->rhocf, c->xcL, c->ycL, c->dxL, c->dyL,
                    c->muX, c->muY, c->muD, c->muA, c->Wx, c->Wy, c->Wc, c->Wpx, c->Wpy,
                    c->Wpc};
  for (size_t a = 0; a < sizeof arrs / sizeof arrs[0]; ++a) free(arrs[a]);
  free(c->pure);
  free(c->flags);
  free(c);
}

const char *lr_ref_last_error(const lr_ref_ctx *c) { return c ? c->err : "null context"; }

/* zero the wall-normal velocity component on wall nodes (reflective walls) */
static void wall_nodes(const lr_ref_ctx *c, double *vx, double *vy) {
  for (int J = 0; J <= c->ny; ++J)
    for (int I = 0; I <= c->nx; ++I) {
      if (I == 0 || I == c->nx) vx[NI(c, I, J)] = 0.0;
      if (J == 0 || J == c->ny) vy[NI(c, I, J)] = 0.0;
    }
}

int lr_ref_set_state(lr_ref_ctx *c, double t, const double *k, const double *rho,
                     const double *e, const double *ux, const double *uy) {
  if (!c || !k || !rho || !e || !ux || !uy) return LR_REF_EINVAL;
  int nx = c->nx, ny = c->ny, nm = c->nmat;
  size_t cells = (size_t)nx * ny;
  if (!isfinite(t)) return fail(c, LR_REF_EINVAL, "t not finite");
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double ks = 0.0;
      for (int a = 0; a < nm; ++a) {
        size_t h = a * cells + (size_t)j * nx + i;
        if (!isfinite(k[h]) || !isfinite(rho[h]) || !isfinite(e[h]))
          return fail(c, LR_REF_ENAN, "non-finite input");
        if (k[h] < 0.0 || k[h] > 1.0) return fail(c, LR_REF_ESTATE, "volume fraction outside [0,1]");
        if (k[h] > 0.0 && (!(rho[h] > 0.0) || e[h] < 0.0))
          return fail(c, LR_REF_ESTATE, "rho <= 0 or e < 0 where k > 0");
        ks += k[h];
      }
      if (fabs(ks - 1.0) > 1e-12) return fail(c, LR_REF_ESTATE, "volume fractions do not sum to 1");
    }
  for (size_t p = 0; p < (size_t)(nx + 1) * (ny + 1); ++p)
    if (!isfinite(ux[p]) || !isfinite(uy[p])) return fail(c, LR_REF_ENAN, "non-finite velocity");
  for (int a = 0; a < nm; ++a)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t h = a * cells + (size_t)j * nx + i;
        int q = a * ncell(c) + CI(c, i, j);
        double V = k[h] * c->A;
        double M = k[h] > 0.0 ? rho[h] * V : 0.0;
        c->V[q] = V;
        c->M[q] = M;
        c->E[q] = k[h] > 0.0 ? M * e[h] : 0.0;
      }
  for (int J = 0; J <= ny; ++J)
    for (int I = 0; I <= nx; ++I) {
      c->ux[NI(c, I, J)] = ux[(size_t)J * (nx + 1) + I];
      c->uy[NI(c, I, J)] = uy[(size_t)J * (nx + 1) + I];
    }
  wall_nodes(c, c->ux, c->uy);
  c->t = t;
  c->step = 0;
  c->have_state = 1;
  memset(c->counts, 0, sizeof c->counts);
  return LR_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* stage: quantities at t^n                                                  */
static int present(const lr_ref_ctx *c, double V) { return V > c->o.k_eps * c->A; }

static void derived(lr_ref_ctx *c) {
  int C = ncell(c);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < c->ny; ++j)
    for (int i = 0; i < c->nx; ++i) {
      int q = CI(c, i, j);
      double Msum = 0.0, Pc = 0.0, rc2 = 0.0;
      for (int a = 0; a < c->nmat; ++a) {
        double V = c->V[a * C + q], M = c->M[a * C + q], E = c->E[a * C + q];
        c->k[a * C + q] = V / c->A;
        if (present(c, V)) {
          double rho = M / V;
          double e = M > 0.0 ? E / M : 0.0;
          double P = eos_p(c, a, rho, e);
          c->rho_a[a * C + q] = rho;
          c->e_a[a * C + q] = e;
          c->P_a[a * C + q] = P;
          Pc += c->k[a * C + q] * P;                  /* §4.1: P_c = sum k P */
          rc2 += eos_k_rho_c2(c, a, c->k[a * C + q], P); /* reading: rho c^2 = sum k rho_a c_a^2 */
        } else {
          c->rho_a[a * C + q] = 0.0;
          c->e_a[a * C + q] = M > 0.0 ? E / M : 0.0;
          c->P_a[a * C + q] = 0.0;
        }
        Msum += M;
      }
      c->Mc[q] = Msum;
      c->rhoc[q] = Msum / c->A;
      c->Pc[q] = Pc;
      double c2 = c->rhoc[q] > 0.0 ? rc2 / c->rhoc[q] : 0.0;
      c->cc[q] = c2 > 0.0 ? sqrt(c2) : 0.0;
    }
  for (int a = 0; a < c->nmat; ++a) {
    ghost_cells(c, c->k + a * C);
    ghost_cells(c, c->rho_a + a * C);
    ghost_cells(c, c->e_a + a * C);
  }
  ghost_cells(c, c->Mc);
  ghost_cells(c, c->rhoc);
  ghost_cells(c, c->cc);
  ghost_cells(c, c->Pc);
}

/* reading: dt = CFL min_c min(dx/(c+max|ux|), dy/(c+max|uy|)) over the four
 * nodes of c, the last step clamped to t_end */
static double cfl_dt(const lr_ref_ctx *c) {
  double *row = dalloc(c->ny);
  if (!row) return NAN;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < c->ny; ++j) {
    double best = INFINITY;
    for (int i = 0; i < c->nx; ++i) {
      double Ux = 0.0, Uy = 0.0;
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          Ux = fmax(Ux, fabs(c->ux[NI(c, i + a, j + b)]));
          Uy = fmax(Uy, fabs(c->uy[NI(c, i + a, j + b)]));
        }
      double cs = c->cc[CI(c, i, j)];
      double cand = fmin(c->dx / (cs + Ux), c->dy / (cs + Uy));
      best = fmin(best, cand);
    }
    row[j] = best;
  }
  double best = INFINITY;
  for (int j = 0; j < c->ny; ++j) best = fmin(best, row[j]);
  free(row);
  return c->o.cfl * best;
}

/* §1.2: discrete Wilkins pseudo-viscosity with Delta u ~ L div u, L = sqrt(dx dy);
 * reading: rho multiplies both terms, div u from the four nodal velocities */
static void pseudo_viscosity(lr_ref_ctx *c) {
  double L = sqrt(c->A);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < c->ny; ++j)
    for (int i = 0; i < c->nx; ++i) {
      double uBLx = c->ux[NI(c, i, j)], uBRx = c->ux[NI(c, i + 1, j)];
      double uTLx = c->ux[NI(c, i, j + 1)], uTRx = c->ux[NI(c, i + 1, j + 1)];
      double uBLy = c->uy[NI(c, i, j)], uBRy = c->uy[NI(c, i + 1, j)];
      double uTLy = c->uy[NI(c, i, j + 1)], uTRy = c->uy[NI(c, i + 1, j + 1)];
      double div = (uBRx + uTRx - uBLx - uTLx) / (2.0 * c->dx) +
                   (uTLy + uTRy - uBLy - uBRy) / (2.0 * c->dy);
      double q = 0.0;
      int cq = CI(c, i, j);
      if (div < 0.0 && !c->o.kinematic)
        q = c->rhoc[cq] * (c->o.a1 * L * c->cc[cq] * fabs(div) + c->o.a2 * L * L * div * div);
      c->Q[cq] = q;
    }
  ghost_cells(c, c->Q);
}

/* §1.2: nodal mass m_p = 1/4 sum of the four cell masses */
static void nodal_mass(lr_ref_ctx *c) {
#pragma omp parallel for schedule(static)
  for (int J = 0; J <= c->ny; ++J)
    for (int I = 0; I <= c->nx; ++I)
      c->mp[NI(c, I, J)] = 0.25 * (c->Mc[CI(c, I - 1, J - 1)] + c->Mc[CI(c, I, J - 1)] +
                                   c->Mc[CI(c, I - 1, J)] + c->Mc[CI(c, I, J)]);
}

/* the quad volume of cell (i,j) when its nodes are displaced by (hx,hy),
 * in coordinates local to the cell's Eulerian bottom-left node */
static double cell_F(const lr_ref_ctx *c, int i, int j, const double *hx, const double *hy) {
  int bl = NI(c, i, j), br = NI(c, i + 1, j), tl = NI(c, i, j + 1), tr = NI(c, i + 1, j + 1);
  return quad_F(hx[bl], hy[bl], c->dx + hx[br], hy[br], hx[tl], c->dy + hy[tl],
                c->dx + hx[tr], c->dy + hy[tr]);
}

/* §1.2 eq. "prediction" with §4.1 eq. "prediction_multi" */
static void predictor(lr_ref_ctx *c, double dt) {
  int C = ncell(c), N = nnode(c);
  double *hx = dalloc(N), *hy = dalloc(N);
#pragma omp parallel for schedule(static)
  for (int J = 0; J <= c->ny; ++J)
    for (int I = 0; I <= c->nx; ++I) {
      int p = NI(c, I, J);
      hx[p] = 0.5 * dt * c->ux[p]; /* x^{n+1/2} - x^n */
      hy[p] = 0.5 * dt * c->uy[p];
    }
#pragma omp parallel for schedule(static)
  for (int j = 0; j < c->ny; ++j)
    for (int i = 0; i < c->nx; ++i) {
      int q = CI(c, i, j);
      double Vh = cell_F(c, i, j, hx, hy); /* Vol_c^{n+1/2} */
      double Pch = 0.0;
      for (int a = 0; a < c->nmat; ++a) {
        int qa = a * C + q;
        double V = c->V[qa], M = c->M[qa];
        if (present(c, V)) {
          double Vah = c->k[qa] * Vh;              /* Vol_a^{n+1/2} = k_a Vol_c^{n+1/2} */
          double rho_h = M / Vah;
          double e_h = c->e_a[qa] - (c->P_a[qa] + c->Q[q]) * (1.0 / rho_h - 1.0 / c->rho_a[qa]);
          double P_h = eos_p(c, a, rho_h, e_h);
          c->e_half[qa] = e_h;
          c->P_half[qa] = P_h;
          Pch += c->k[qa] * P_h;
        } else {
          c->e_half[qa] = c->e_a[qa];
          c->P_half[qa] = 0.0;
        }
      }
      c->Pc_half[q] = Pch;
      c->S[q] = Pch + c->Q[q]; /* P^{n+1/2} + Q^n */
    }
  ghost_cells(c, c->S);
  /* nodal gradient of P+Q and velocity prediction */
#pragma omp parallel for schedule(static)
  for (int J = 0; J <= c->ny; ++J)
    for (int I = 0; I <= c->nx; ++I) {
      int p = NI(c, I, J);
      double sSW = c->S[CI(c, I - 1, J - 1)], sSE = c->S[CI(c, I, J - 1)];
      double sNW = c->S[CI(c, I - 1, J)], sNE = c->S[CI(c, I, J)];
      double gx = ((sSE + sNE) - (sSW + sNW)) / (2.0 * c->dx);
      double gy = ((sNW + sNE) - (sSW + sSE)) / (2.0 * c->dy);
      double rho_p = c->mp[p] / c->A;
      c->uhx[p] = c->ux[p] - 0.5 * dt * gx / rho_p;
      c->uhy[p] = c->uy[p] - 0.5 * dt * gy / rho_p;
    }
  wall_nodes(c, c->uhx, c->uhy);
  free(hx);
  free(hy);
}

/* §1.2 eq. "correction" with §4.1 eq. "correction_multi" */
static void corrector(lr_ref_ctx *c, double dt) {
  int C = ncell(c);
#pragma omp parallel for schedule(static)
  for (int J = 0; J <= c->ny; ++J)
    for (int I = 0; I <= c->nx; ++I) {
      int p = NI(c, I, J);
      c->dpx[p] = dt * c->uhx[p]; /* x^{lag} - x^n */
      c->dpy[p] = dt * c->uhy[p];
      c->uLx[p] = 2.0 * c->uhx[p] - c->ux[p];
      c->uLy[p] = 2.0 * c->uhy[p] - c->uy[p];
    }
  wall_nodes(c, c->uLx, c->uLy);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < c->ny; ++j)
    for (int i = 0; i < c->nx; ++i) {
      int q = CI(c, i, j);
      double VL = cell_F(c, i, j, c->dpx, c->dpy); /* Vol_c^{n+1,lag} */
      c->VL[q] = VL;
      for (int a = 0; a < c->nmat; ++a) {
        int qa = a * C + q;
        if (present(c, c->V[qa])) {
          double rho_L = c->M[qa] / (c->k[qa] * VL);
          c->eL[qa] = c->e_a[qa] - (c->P_half[qa] + c->Q[q]) * (1.0 / rho_L - 1.0 / c->rho_a[qa]);
        } else {
          c->eL[qa] = c->e_a[qa];
        }
      }
    }
}

/* prescribed node velocities (tests of the remap alone, §5.1 rotation cases) */
static void kinematic_lagrange(lr_ref_ctx *c, double dt) {
  int C = ncell(c);
  for (int J = 0; J <= c->ny; ++J)
    for (int I = 0; I <= c->nx; ++I) {
      int p = NI(c, I, J);
      c->uhx[p] = c->ux[p]; c->uhy[p] = c->uy[p];
      c->uLx[p] = c->ux[p]; c->uLy[p] = c->uy[p];
      c->dpx[p] = dt * c->ux[p]; c->dpy[p] = dt * c->uy[p];
    }
  for (int j = 0; j < c->ny; ++j)
    for (int i = 0; i < c->nx; ++i) {
      int q = CI(c, i, j);
      c->VL[q] = cell_F(c, i, j, c->dpx, c->dpy);
      for (int a = 0; a < c->nmat; ++a) c->eL[a * C + q] = c->e_a[a * C + q];
    }
}

/* ------------------------------------------------------------------------ */
/* remap regions                                                             */
/* A region is one face or corner flux volume: a rectangle, its volume, the
 * donor and receiver cells, and the sign of the flux along its orientation
 * (+x for x-faces, +y for y-faces, SW->NE for main-diagonal corners and
 * NW->SE for anti-diagonal corners). */
typedef struct {
  double vol;                /* |dVol| */
  double rx0, rx1, ry0, ry1; /* flux rectangle, relative to Eulerian node (I,J) */
  int di, dj, ri, rj;        /* donor, receiver */
  double sgn;                /* +1: flux along the orientation */
  int type;                  /* 0 x-face, 1 y-face, 2 corner main, 3 corner anti */
  int I, J;                  /* face / node index */
  double W[LR_REF_MAXMAT], mu[LR_REF_MAXMAT], eps[LR_REF_MAXMAT];
  double vrho[LR_REF_MAXMAT], ve[LR_REF_MAXMAT];
} region;

/* §2.3: corner volume flux at node (I,J): |dx dy|, donor and receiver from the
 * signs of the node displacement (§3.3 upwind table) */
static void corner_region(const lr_ref_ctx *c, int I, int J, region *r) {
  memset(r, 0, sizeof *r);
  int p = NI(c, I, J);
  double dx = c->dpx[p], dy = c->dpy[p];
  r->vol = fabs(dx * dy);
  r->I = I; r->J = J;
  int sx = dx >= 0.0, sy = dy >= 0.0;
  if (sx && sy) { r->type = 2; r->di = I - 1; r->dj = J - 1; r->ri = I; r->rj = J; r->sgn = 1; }
  else if (!sx && !sy) { r->type = 2; r->di = I; r->dj = J; r->ri = I - 1; r->rj = J - 1; r->sgn = -1; }
  else if (sx && !sy) { r->type = 3; r->di = I - 1; r->dj = J; r->ri = I; r->rj = J - 1; r->sgn = 1; }
  else { r->type = 3; r->di = I; r->dj = J - 1; r->ri = I - 1; r->rj = J; r->sgn = -1; }
  r->rx0 = fmin(0.0, dx); r->rx1 = fmax(0.0, dx);
  r->ry0 = fmin(0.0, dy); r->ry1 = fmax(0.0, dy);
}

/* §2.3: x-face (I,j) flux: the trapezoid between the Eulerian face and the
 * Lagrangian face line, cut at y_f^- = y_{p-} + max(0,dy_{p-}) and
 * y_f^+ = y_{p+} + min(0,dy_{p+}), replaced by the rectangle of the same area
 * (reading: x_f^+- are signed offsets of the Lagrangian line from the face) */
static void xface_region(const lr_ref_ctx *c, int I, int j, region *r) {
  memset(r, 0, sizeof *r);
  int pm = NI(c, I, j), pp = NI(c, I, j + 1);
  /* local coordinates: origin at the face's Eulerian lower node */
  double xm = c->dpx[pm], ym = c->dpy[pm];             /* x^{lag}_{p-} */
  double xp = c->dpx[pp], yp = c->dy + c->dpy[pp];     /* x^{lag}_{p+} */
  double ylo = fmax(0.0, c->dpy[pm]);
  double yhi = c->dy + fmin(0.0, c->dpy[pp]);
  double h = yhi - ylo;
  if (h < 0.0) h = 0.0;
  double slope = (xp - xm) / (yp - ym);
  double xlo = xm + (ylo - ym) * slope;
  double xhi = xm + (yhi - ym) * slope;
  double w = 0.5 * (xlo + xhi);
  double W = w * h;
  r->type = 0; r->I = I; r->J = j;
  r->vol = fabs(W);
  if (w >= 0.0) { r->di = I - 1; r->dj = j; r->ri = I; r->rj = j; r->sgn = 1; }
  else { r->di = I; r->dj = j; r->ri = I - 1; r->rj = j; r->sgn = -1; }
  r->rx0 = fmin(0.0, w); r->rx1 = fmax(0.0, w);
  r->ry0 = ylo; r->ry1 = ylo + h;
}

/* same for the y-face (i,J) with x and y exchanged */
static void yface_region(const lr_ref_ctx *c, int i, int J, region *r) {
  memset(r, 0, sizeof *r);
  int pm = NI(c, i, J), pp = NI(c, i + 1, J);
  double xm = c->dpx[pm], ym = c->dpy[pm];
  double xp = c->dx + c->dpx[pp], yp = c->dpy[pp];
  double xlo = fmax(0.0, c->dpx[pm]);
  double xhi = c->dx + fmin(0.0, c->dpx[pp]);
  double h = xhi - xlo;
  if (h < 0.0) h = 0.0;
  double slope = (yp - ym) / (xp - xm);
  double ylo = ym + (xlo - xm) * slope;
  double yhi = ym + (xhi - xm) * slope;
  double w = 0.5 * (ylo + yhi);
  double W = w * h;
  r->type = 1; r->I = i; r->J = J;
  r->vol = fabs(W);
  if (w >= 0.0) { r->di = i; r->dj = J - 1; r->ri = i; r->rj = J; r->sgn = 1; }
  else { r->di = i; r->dj = J; r->ri = i; r->rj = J - 1; r->sgn = -1; }
  r->rx0 = xlo; r->rx1 = xlo + h;
  r->ry0 = fmin(0.0, w); r->ry1 = fmax(0.0, w);
}

/* The eight regions touching cell (i,j) in the fixed order W, E, S, N faces
 * then BL, BR, TL, TR corners (reading: the summation order). */
typedef struct { region *r; } regref;

typedef struct {
  region *xf, *yf, *cn; /* real faces and corners */
} regions;

static region *XF(const lr_ref_ctx *c, regions *R, int I, int j) { return &R->xf[j * (c->nx + 1) + I]; }
static region *YF(const lr_ref_ctx *c, regions *R, int i, int J) { return &R->yf[J * c->nx + i]; }
static region *CN(const lr_ref_ctx *c, regions *R, int I, int J) { return &R->cn[J * (c->nx + 1) + I]; }

static void cell_regions(const lr_ref_ctx *c, regions *R, int i, int j, region *out[8]) {
  out[0] = XF(c, R, i, j);
  out[1] = XF(c, R, i + 1, j);
  out[2] = YF(c, R, i, j);
  out[3] = YF(c, R, i, j + 1);
  out[4] = CN(c, R, i, j);
  out[5] = CN(c, R, i + 1, j);
  out[6] = CN(c, R, i, j + 1);
  out[7] = CN(c, R, i + 1, j + 1);
}
static int is_donor(const region *r, int i, int j) { return r->di == i && r->dj == j; }
static int is_receiver(const region *r, int i, int j) { return r->ri == i && r->rj == j; }

/* Youngs normal gradient of k_a on the 3x3 block (reading: 1-2-1 weights) */
static void youngs(const lr_ref_ctx *c, int a, int i, int j, double *gx, double *gy) {
  const double *k = c->k + a * ncell(c);
#define K(ii, jj) k[CI(c, ii, jj)]
  *gx = ((K(i + 1, j - 1) + 2.0 * K(i + 1, j) + K(i + 1, j + 1)) -
         (K(i - 1, j - 1) + 2.0 * K(i - 1, j) + K(i - 1, j + 1))) / (8.0 * c->dx);
  *gy = ((K(i - 1, j + 1) + 2.0 * K(i, j + 1) + K(i + 1, j + 1)) -
         (K(i - 1, j - 1) + 2.0 * K(i, j - 1) + K(i + 1, j - 1))) / (8.0 * c->dy);
#undef K
}

/* §4.4: the rectangular approximation of the Lagrangian cell (i,j), through
 * the midpoints of its four Lagrangian faces, in coordinates local to the
 * Eulerian cell centre.  mx, my = 0 keep that direction's faces Eulerian (the
 * X- and Y-Lagrangian cells of the alternate-direction remap, §4.2). */
static void lagrangian_rectangle(const lr_ref_ctx *c, int i, int j, int mx, int my,
                                 double *Rx0, double *Rx1, double *Ry0, double *Ry1) {
  int bl = NI(c, i, j), br = NI(c, i + 1, j), tl = NI(c, i, j + 1), tr = NI(c, i + 1, j + 1);
  *Rx0 = (mx ? 0.5 * (c->dpx[bl] + c->dpx[tl]) : 0.0) - 0.5 * c->dx;
  *Rx1 = (mx ? 0.5 * (c->dpx[br] + c->dpx[tr]) : 0.0) + 0.5 * c->dx;
  *Ry0 = (my ? 0.5 * (c->dpy[bl] + c->dpy[br]) : 0.0) - 0.5 * c->dy;
  *Ry1 = (my ? 0.5 * (c->dpy[tl] + c->dpy[tr]) : 0.0) + 0.5 * c->dy;
}

/* §4.4: split every outflow region of mixed donor (i,j) (rs[0..nr-1], the
 * regions touching it) between its present materials with the interface
 * placed on the rectangle R of its Lagrangian cell, then the donor-side
 * clipping (reading) against k_a vlag, vlag its flux-consistent Lagrangian
 * volume. */
static void mixed_donor_partials(lr_ref_ctx *c, region **rs, int nr, int i, int j,
                                 double Rx0, double Rx1, double Ry0, double Ry1,
                                 double vlag) {
  int C = ncell(c), q = CI(c, i, j), nm = c->nmat;
  int pres[LR_REF_MAXMAT], np = 0;
  double Vp = 0.0;
  for (int a = 0; a < nm; ++a) {
    pres[a] = present(c, c->V[a * C + q]);
    if (pres[a]) { ++np; Vp += c->V[a * C + q]; }
  }
  /* reading: a Youngs gradient below gmin is numerical noise -> no normal */
  double gmin = 1e-10 / fmin(c->dx, c->dy);

  double nxv[LR_REF_MAXMAT], nyv[LR_REF_MAXMAT], sv[LR_REF_MAXMAT];
  int degenerate = 0, a0 = -1, b0 = -1;
  c->flags[q] |= F_MIXED | (np >= 3 ? F_THREE : 0);
  if (np == 2) {
    for (int a = 0; a < nm; ++a)
      if (pres[a]) { if (a0 < 0) a0 = a; else b0 = a; }
    double gax, gay, gbx, gby;
    youngs(c, a0, i, j, &gax, &gay);
    youngs(c, b0, i, j, &gbx, &gby);
    double gx = gax - gbx, gy = gay - gby;
    double nrm = sqrt(gx * gx + gy * gy);
    if (nrm <= gmin) degenerate = 1;
    else {
      nxv[a0] = gx / nrm; nyv[a0] = gy / nrm;
      sv[a0] = lr_ref_interface_offset(Rx0, Rx1, Ry0, Ry1, nxv[a0], nyv[a0],
                                       c->V[a0 * C + q] / Vp);
    }
  } else {
    for (int a = 0; a < nm; ++a) {
      if (!pres[a]) continue;
      double gx, gy;
      youngs(c, a, i, j, &gx, &gy);
      double nrm = sqrt(gx * gx + gy * gy);
      if (nrm <= gmin) { degenerate = 1; continue; }
      nxv[a] = gx / nrm; nyv[a] = gy / nrm;
      sv[a] = lr_ref_interface_offset(Rx0, Rx1, Ry0, Ry1, nxv[a], nyv[a], c->V[a * C + q] / Vp);
    }
  }
  if (degenerate) c->flags[q] |= F_DEGENERATE;
  /* partial volumes of each outflow region */
  for (int s = 0; s < nr; ++s) {
    region *r = rs[s];
    if (!is_donor(r, i, j)) continue;
    for (int a = 0; a < nm; ++a) r->W[a] = 0.0;
    if (r->vol == 0.0) continue;
    /* region rectangle moved to the donor-centred frame: its origin node
     * (I,J) sits at ((I-i-1/2) dx, (J-j-1/2) dy) from the centre of (i,j) */
    double ox = ((r->I - i) - 0.5) * c->dx, oy = ((r->J - j) - 0.5) * c->dy;
    double x0 = r->rx0 + ox, x1 = r->rx1 + ox, y0 = r->ry0 + oy, y1 = r->ry1 + oy;
    if (degenerate) {
      /* reading: no usable normal -> split in proportion to the volumes */
      for (int a = 0; a < nm; ++a)
        if (pres[a]) r->W[a] = r->vol * (c->V[a * C + q] / Vp);
    } else if (np == 2) {
      double wa = lr_ref_rect_halfplane_area(x0, x1, y0, y1, nxv[a0], nyv[a0], sv[a0]);
      if (wa < 0.0) wa = 0.0;
      if (wa > r->vol) wa = r->vol;
      r->W[a0] = wa;
      r->W[b0] = r->vol - wa;
    } else {
      /* reading: three or more materials, one line each, normalised */
      double raw[LR_REF_MAXMAT], sum = 0.0;
      for (int a = 0; a < nm; ++a) {
        raw[a] = pres[a] ? lr_ref_rect_halfplane_area(x0, x1, y0, y1, nxv[a], nyv[a], sv[a]) : 0.0;
        sum += raw[a];
      }
      for (int a = 0; a < nm; ++a) {
        if (!pres[a]) continue;
        r->W[a] = sum > 0.0 ? r->vol * (raw[a] / sum) : r->vol * (c->V[a * C + q] / Vp);
      }
    }
  }
  /* reading: donor-side limiting so that no material sends more volume than
   * its flux-consistent Lagrangian volume; the excess goes to the donor's
   * other materials in proportion to their remaining room */
  double Vcf[LR_REF_MAXMAT], O[LR_REF_MAXMAT];
  int over[LR_REF_MAXMAT], any_over = 0;
  for (int a = 0; a < nm; ++a) {
    Vcf[a] = c->k[a * C + q] * vlag;
    O[a] = 0.0;
    for (int s = 0; s < nr; ++s)
      if (is_donor(rs[s], i, j)) O[a] += rs[s]->W[a];
    over[a] = pres[a] && O[a] > Vcf[a];
    any_over |= over[a];
  }
  if (!any_over) return;
  double room[LR_REF_MAXMAT], H = 0.0;
  for (int a = 0; a < nm; ++a) {
    room[a] = (pres[a] && !over[a]) ? fmax(0.0, Vcf[a] - O[a]) : 0.0;
    H += room[a];
  }
  if (!(H > 0.0)) return;
  c->flags[q] |= F_CLIPPED;
  for (int s = 0; s < nr; ++s) {
    region *r = rs[s];
    if (!is_donor(r, i, j)) continue;
    double freed = 0.0;
    for (int a = 0; a < nm; ++a)
      if (over[a]) {
        double keep = r->W[a] * (Vcf[a] / O[a]);
        freed += r->W[a] - keep;
        r->W[a] = keep;
      }
    for (int a = 0; a < nm; ++a)
      if (room[a] > 0.0) r->W[a] += freed * (room[a] / H);
  }
}

/* one-sided slopes along a direction between Lagrangian centres, limited */
static double slope_dir(const lr_ref_ctx *c, const double *a, int i, int j, int si, int sj,
                        double vx, double vy) {
  int q = CI(c, i, j), qm = CI(c, i - si, j - sj), qp = CI(c, i + si, j + sj);
  double dm = (a[q] - a[qm]) / ((c->xcL[q] - c->xcL[qm]) * vx + (c->ycL[q] - c->ycL[qm]) * vy);
  double dp = (a[qp] - a[q]) / ((c->xcL[qp] - c->xcL[q]) * vx + (c->ycL[qp] - c->ycL[q]) * vy);
  return van_leer(dm, dp);
}

/* reading: second order only if the donor and both neighbours along the
 * reconstruction direction are pure cells of the donor's material */
static int stencil_pure(const lr_ref_ctx *c, int i, int j, int si, int sj) {
  int m = c->pure[CI(c, i, j)];
  return m >= 0 && c->pure[CI(c, i - si, j - sj)] == m && c->pure[CI(c, i + si, j + sj)] == m;
}

/* §3.3, multidimensional reconstruction: the plane a_D + G.(x - x_D) over the
 * 3 x 3 stencil, its gradient G the least-squares fit of the eight
 * neighbours' values at their Lagrangian centres (the normal equations of
 * the 2 x 2 system, solved by the cofactor formula), scaled by
 * phi = min(|d_x|, |d_y|, |d_v|, |d_vperp|) / |G| with the four limited
 * one-dimensional slopes, and evaluated at the centre of the region's flux
 * rectangle.  Readings: order 2 only if all nine cells are pure cells of
 * the donor's material; a degenerate fit or G = 0 gives the donor's value. */
static double recon_lsq(const lr_ref_ctx *c, const region *r, const double *arr) {
  int i = r->di, j = r->dj, q = CI(c, i, j);
  double aD = arr[q];
  int m = c->pure[q];
  if (m < 0) return aD;
  for (int b = -1; b <= 1; ++b)
    for (int a = -1; a <= 1; ++a)
      if (c->pure[CI(c, i + a, j + b)] != m) return aD;
  double s11 = 0.0, s12 = 0.0, s22 = 0.0, b1 = 0.0, b2 = 0.0;
  for (int b = -1; b <= 1; ++b)
    for (int a = -1; a <= 1; ++a) {
      if (a == 0 && b == 0) continue;
      int k = CI(c, i + a, j + b);
      double X1 = c->xcL[k] - c->xcL[q], X2 = c->ycL[k] - c->ycL[q], A = arr[k] - aD;
      s11 += X1 * X1; s12 += X1 * X2; s22 += X2 * X2;
      b1 += X1 * A; b2 += X2 * A;
    }
  double det = s11 * s22 - s12 * s12;
  if (!(det > 0.0)) return aD;
  double G1 = (s22 * b1 - s12 * b2) / det, G2 = (s11 * b2 - s12 * b1) / det;
  double nG = sqrt(G1 * G1 + G2 * G2);
  if (!(nG > 0.0)) return aD;
  double nrm = sqrt(c->dx * c->dx + c->dy * c->dy);
  double lim = fabs(slope_dir(c, arr, i, j, 1, 0, 1.0, 0.0));
  lim = fmin(lim, fabs(slope_dir(c, arr, i, j, 0, 1, 0.0, 1.0)));
  lim = fmin(lim, fabs(slope_dir(c, arr, i, j, 1, 1, c->dx / nrm, c->dy / nrm)));
  lim = fmin(lim, fabs(slope_dir(c, arr, i, j, 1, -1, c->dx / nrm, -c->dy / nrm)));
  double phi = lim / nG;
  double xr = node_x(c, r->I) + 0.5 * (r->rx0 + r->rx1);
  double yr = node_y(c, r->J) + 0.5 * (r->ry0 + r->ry1);
  return aD + phi * (G1 * (xr - c->xcL[q]) + G2 * (yr - c->ycL[q]));
}

/* §2.1.1 and §3.3: value of a donor quantity on region r at order 1, 2
 * (limited linear along the region's direction) or 3 (multidimensional) */
static double recon(const lr_ref_ctx *c, const region *r, const double *arr, int order) {
  int i = r->di, j = r->dj, q = CI(c, i, j);
  double aD = arr[q];
  if (order == 1) return aD;
  if (order == 3) return recon_lsq(c, r, arr);
  if (r->type == 0) {
    if (!stencil_pure(c, i, j, 1, 0)) return aD;
    double d = slope_dir(c, arr, i, j, 1, 0, 1.0, 0.0);
    /* sgn(dVol) dx^{lag}_c - dt u_f, u_f the mean of the face's two nodes */
    double uf = 0.5 * (c->dpx[NI(c, r->I, r->J)] + c->dpx[NI(c, r->I, r->J + 1)]);
    return aD + 0.5 * d * (r->sgn * c->dxL[q] - uf);
  }
  if (r->type == 1) {
    if (!stencil_pure(c, i, j, 0, 1)) return aD;
    double d = slope_dir(c, arr, i, j, 0, 1, 0.0, 1.0);
    double uf = 0.5 * (c->dpy[NI(c, r->I, r->J)] + c->dpy[NI(c, r->I + 1, r->J)]);
    return aD + 0.5 * d * (r->sgn * c->dyL[q] - uf);
  }
  double nrm = sqrt(c->dx * c->dx + c->dy * c->dy);
  int p = NI(c, r->I, r->J);
  double sx = c->dpx[p] >= 0.0 ? 1.0 : -1.0; /* sgn(dx_p) */
  if (r->type == 2) {
    if (!stencil_pure(c, i, j, 1, 1)) return aD;
    double vx = c->dx / nrm, vy = c->dy / nrm;
    double d = slope_dir(c, arr, i, j, 1, 1, vx, vy);
    double off = (sx * c->dxL[q] - c->dpx[p]) * vx + (sx * c->dyL[q] - c->dpy[p]) * vy;
    return aD + 0.5 * d * off;
  }
  if (!stencil_pure(c, i, j, 1, -1)) return aD;
  double vx = c->dx / nrm, vy = -c->dy / nrm;
  double d = slope_dir(c, arr, i, j, 1, -1, vx, vy);
  double off = (sx * c->dxL[q] - c->dpx[p]) * vx + (-sx * c->dyL[q] - c->dpy[p]) * vy;
  return aD + 0.5 * d * off;
}

/* ------------------------------------------------------------------------ */
/* dual mesh (momentum) reconstruction, reading: the same 1D/diagonal rules on
 * the dual mesh, dual centres at the Lagrangian node positions, dual widths
 * dx + (d_{I+1} - d_{I-1})/2, dual face displacement the mean of its two nodes,
 * dual corner displacement the mean of the cell's four nodes. */
static double dual_slope(const lr_ref_ctx *c, const double *u, int I, int J, int sI, int sJ,
                         double vx, double vy) {
  int p = NI(c, I, J), pm = NI(c, I - sI, J - sJ), pp = NI(c, I + sI, J + sJ);
  double dm = (u[p] - u[pm]) / ((c->xLx[p] - c->xLx[pm]) * vx + (c->xLy[p] - c->xLy[pm]) * vy);
  double dp = (u[pp] - u[p]) / ((c->xLx[pp] - c->xLx[p]) * vx + (c->xLy[pp] - c->xLy[p]) * vy);
  return van_leer(dm, dp);
}
static double dual_wx(const lr_ref_ctx *c, int I, int J) {
  return c->dx + 0.5 * (c->dpx[NI(c, I + 1, J)] - c->dpx[NI(c, I - 1, J)]);
}
static double dual_wy(const lr_ref_ctx *c, int I, int J) {
  return c->dy + 0.5 * (c->dpy[NI(c, I, J + 1)] - c->dpy[NI(c, I, J - 1)]);
}

/* outflow partial volumes of donor (i,j): a pure donor sends its material
 * only, a mixed one is split by its interface (§4.4) */
static void donor_partials(lr_ref_ctx *c, region **rs, int nr, int i, int j, int mx, int my,
                           double vlag) {
  int q = CI(c, i, j), nm = c->nmat;
  if (c->pure[q] >= 0) {
    for (int s = 0; s < nr; ++s)
      if (is_donor(rs[s], i, j)) {
        for (int a = 0; a < nm; ++a) rs[s]->W[a] = 0.0;
        rs[s]->W[c->pure[q]] = rs[s]->vol;
      }
  } else {
    double Rx0, Rx1, Ry0, Ry1;
    lagrangian_rectangle(c, i, j, mx, my, &Rx0, &Rx1, &Ry0, &Ry1);
    mixed_donor_partials(c, rs, nr, i, j, Rx0, Rx1, Ry0, Ry1, vlag);
  }
}

/* reconstruction and mass / energy fluxes of the outflow regions of donor
 * (i,j) (§2.1.1, §3.3, §4.2) */
static void donor_fluxes(lr_ref_ctx *c, region **rs, int nr, int i, int j) {
  int C = ncell(c), q = CI(c, i, j), nm = c->nmat;
  int order = c->o.recon_order;
  if (c->pure[q] < 0) order = 1; /* §4.2: mixed donors degenerate to order 1 */
  for (int pass = 0; pass < 2; ++pass) {
    double Mout[LR_REF_MAXMAT] = {0}, Eout[LR_REF_MAXMAT] = {0};
    for (int s = 0; s < nr; ++s) {
      region *r = rs[s];
      if (!is_donor(r, i, j)) continue;
      for (int a = 0; a < nm; ++a) {
        r->mu[a] = r->eps[a] = r->vrho[a] = r->ve[a] = 0.0;
        if (!(r->W[a] > 0.0)) continue;
        double rho = recon(c, r, c->rhocf + a * C, order);
        double e = recon(c, r, c->eL + a * C, order);
        r->vrho[a] = rho;
        r->ve[a] = e;
        r->mu[a] = rho * r->W[a];
        r->eps[a] = r->mu[a] * e;
        Mout[a] += r->mu[a];
        Eout[a] += r->eps[a];
      }
    }
    if (order == 1) break;
    /* reading: positivity guard on the donor's (single present) material:
     * if its order-2 outflow exceeds its mass or Lagrangian internal
     * energy, the whole donor falls back to order 1 */
    int a = c->pure[q], qa = a * C + q;
    if (!(Mout[a] > c->M[qa] || Eout[a] > c->M[qa] * c->eL[qa])) break;
    order = 1;
    c->flags[q] |= F_GUARD;
  }
}

/* conservative update of cell (i,j) from its regions in the order given
 * (§2.3, §4.4): V = k vlag + in - out, M = M + in - out, E = M e^lag + in - out */
static void primal_update(lr_ref_ctx *c, region **rs, int nr, int i, int j, double vlag) {
  int C = ncell(c), q = CI(c, i, j), nm = c->nmat;
  for (int a = 0; a < nm; ++a) {
    int qa = a * C + q;
    double V = c->k[qa] * vlag;
    double M = c->M[qa];
    double E = c->M[qa] * c->eL[qa];
    for (int s = 0; s < nr; ++s) {
      region *r = rs[s];
      if (is_receiver(r, i, j)) { V += r->W[a]; M += r->mu[a]; E += r->eps[a]; }
      else if (is_donor(r, i, j)) { V -= r->W[a]; M -= r->mu[a]; E -= r->eps[a]; }
    }
    c->V[qa] = V;
    c->M[qa] = M;
    c->E[qa] = E;
  }
}

/* §2.3 DirectCF remap of the Lagrangian state: face and corner regions, the
 * flux-consistent Lagrangian volume, partial volumes, reconstruction, primal
 * update, then the dual (momentum) update.  Returns LR_REF_OK or the error
 * code of the last failed check. */
static int remap_directcf(lr_ref_ctx *c) {
  int C = ncell(c), N = nnode(c), nm = c->nmat, nx = c->nx, ny = c->ny;
  int rc = LR_REF_OK;
  /* remap geometry: corner and face volume fluxes (§2.3) */
  regions R;
  R.xf = (region *)calloc((size_t)(nx + 1) * ny, sizeof(region));
  R.yf = (region *)calloc((size_t)nx * (ny + 1), sizeof(region));
  R.cn = (region *)calloc((size_t)(nx + 1) * (ny + 1), sizeof(region));
  if (!R.xf || !R.yf || !R.cn) {
    free(R.xf); free(R.yf); free(R.cn);
    return fail(c, LR_REF_ENOMEM, "out of memory");
  }
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int I = 0; I <= nx; ++I) xface_region(c, I, j, XF(c, &R, I, j));
#pragma omp parallel for schedule(static)
  for (int J = 0; J <= ny; ++J)
    for (int i = 0; i < nx; ++i) yface_region(c, i, J, YF(c, &R, i, J));
#pragma omp parallel for schedule(static)
  for (int J = 0; J <= ny; ++J)
    for (int I = 0; I <= nx; ++I) corner_region(c, I, J, CN(c, &R, I, J));

  /* flux-consistent Lagrangian volume (reading: + outflow - inflow), the
   * Lagrangian cell centre and widths, purity */
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int q = CI(c, i, j);
      region *rs[8];
      cell_regions(c, &R, i, j, rs);
      double v = c->A;
      for (int s = 0; s < 8; ++s) {
        if (is_donor(rs[s], i, j)) v += rs[s]->vol;
        else if (is_receiver(rs[s], i, j)) v -= rs[s]->vol;
      }
      c->volcf[q] = v;
      if (!(v > 0.0)) bad = 1;
      int bl = NI(c, i, j), br = NI(c, i + 1, j), tl = NI(c, i, j + 1), tr = NI(c, i + 1, j + 1);
      c->xcL[q] = 0.25 * (c->xLx[bl] + c->xLx[br] + c->xLx[tl] + c->xLx[tr]);
      c->ycL[q] = 0.25 * (c->xLy[bl] + c->xLy[br] + c->xLy[tl] + c->xLy[tr]);
      c->dxL[q] = c->dx + 0.5 * ((c->dpx[br] + c->dpx[tr]) - (c->dpx[bl] + c->dpx[tl]));
      c->dyL[q] = c->dy + 0.5 * ((c->dpy[tl] + c->dpy[tr]) - (c->dpy[bl] + c->dpy[br]));
      int np = 0, m = -1;
      for (int a = 0; a < nm; ++a) {
        int qa = a * C + q;
        if (present(c, c->V[qa])) { ++np; m = a; }
        /* rho^{lagCF} = m / (k Vol^{lagCF}), e^{lagCF} = e^{lag} (§2.3, §4.4) */
        c->rhocf[qa] = present(c, c->V[qa]) ? c->M[qa] / (c->k[qa] * v) : 0.0;
      }
      c->pure[q] = np == 1 ? m : -1;
    }
  if (bad) rc = fail(c, LR_REF_ENEGATIVE, "flux-consistent Lagrangian volume <= 0");
  for (int a = 0; a < nm; ++a) {
    ghost_cells(c, c->rhocf + a * C);
    ghost_cells(c, c->eL + a * C);
  }
  ghost_cells(c, c->volcf);
  ghost_cells_coord(c, c->xcL, 0);
  ghost_cells_coord(c, c->ycL, 1);
  ghost_cells(c, c->dxL);
  ghost_cells(c, c->dyL);
  ghost_cells_int(c, c->pure);

  /* partial volumes (§4.4) */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      region *rs[8];
      cell_regions(c, &R, i, j, rs);
      donor_partials(c, rs, 8, i, j, 1, 1, c->volcf[CI(c, i, j)]);
    }

  /* reconstruction and mass / energy fluxes, donor by donor */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      region *rs[8];
      cell_regions(c, &R, i, j, rs);
      donor_fluxes(c, rs, 8, i, j);
    }

  /* primal update (§2.3, §4.4), regions in the order W, E, S, N, BL, BR, TL, TR */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      region *rs[8];
      cell_regions(c, &R, i, j, rs);
      primal_update(c, rs, 8, i, j, c->volcf[CI(c, i, j)]);
    }

  /* signed total mass fluxes of every region, then their mirrors */
  for (int p = 0; p < nxf(c); ++p) { c->muX[p] = 0; c->Wx[p] = 0; }
  for (int p = 0; p < nyf(c); ++p) { c->muY[p] = 0; c->Wy[p] = 0; }
  for (int p = 0; p < N; ++p) { c->muD[p] = 0; c->muA[p] = 0; c->Wc[p] = 0; }
  for (int j = 0; j < ny; ++j)
    for (int I = 0; I <= nx; ++I) {
      region *r = XF(c, &R, I, j);
      double m = 0.0;
      for (int a = 0; a < nm; ++a) {
        m += r->mu[a];
        c->Wpx[a * nxf(c) + XI(c, I, j)] = r->sgn * r->W[a];
      }
      c->muX[XI(c, I, j)] = r->sgn * m;
      c->Wx[XI(c, I, j)] = r->sgn * r->vol;
    }
  for (int J = 0; J <= ny; ++J)
    for (int i = 0; i < nx; ++i) {
      region *r = YF(c, &R, i, J);
      double m = 0.0;
      for (int a = 0; a < nm; ++a) {
        m += r->mu[a];
        c->Wpy[a * nyf(c) + YI(c, i, J)] = r->sgn * r->W[a];
      }
      c->muY[YI(c, i, J)] = r->sgn * m;
      c->Wy[YI(c, i, J)] = r->sgn * r->vol;
    }
  for (int J = 0; J <= ny; ++J)
    for (int I = 0; I <= nx; ++I) {
      region *r = CN(c, &R, I, J);
      double m = 0.0;
      for (int a = 0; a < nm; ++a) {
        m += r->mu[a];
        c->Wpc[a * N + NI(c, I, J)] = r->sgn * r->W[a];
      }
      if (r->type == 2) c->muD[NI(c, I, J)] = r->sgn * m;
      else c->muA[NI(c, I, J)] = r->sgn * m;
      c->Wc[NI(c, I, J)] = r->sgn * r->vol;
    }
  free(R.xf); free(R.yf); free(R.cn);
  /* mirrors: an x-mirror negates x fluxes and maps (diag, anti) -> (-anti, -diag);
   * a y-mirror negates y fluxes and maps (diag, anti) -> (anti, diag) */
  for (int j = -G; j < ny + G; ++j)
    for (int I = -G; I <= nx + G; ++I) {
      int rI = mn(I, nx), rj = mc(j, ny);
      if (rI == I && rj == j) continue;
      c->muX[XI(c, I, j)] = (rI != I ? -1.0 : 1.0) * c->muX[XI(c, rI, rj)];
    }
  for (int J = -G; J <= ny + G; ++J)
    for (int i = -G; i < nx + G; ++i) {
      int ri = mc(i, nx), rJ = mn(J, ny);
      if (ri == i && rJ == J) continue;
      c->muY[YI(c, i, J)] = (rJ != J ? -1.0 : 1.0) * c->muY[YI(c, ri, rJ)];
    }
  for (int J = -G; J <= ny + G; ++J)
    for (int I = -G; I <= nx + G; ++I) {
      int rI = mn(I, nx), rJ = mn(J, ny);
      if (rI == I && rJ == J) continue;
      double d = c->muD[NI(c, rI, rJ)], a = c->muA[NI(c, rI, rJ)];
      if (rJ != J) { double t = d; d = a; a = t; }
      if (rI != I) { double t = d; d = -a; a = -t; }
      c->muD[NI(c, I, J)] = d;
      c->muA[NI(c, I, J)] = a;
    }

  /* dual remap of the nodal momentum (§2.1.1 dual mesh, §2.3 dual corners);
   * reading: with the multidimensional reconstruction (order 3) of the cell
   * quantities, the velocities keep the limited linear one along each
   * direction */
  if (!c->o.kinematic) {
    int order = c->o.recon_order;
    double nrm = sqrt(c->dx * c->dx + c->dy * c->dy);
    /* dual x-face (I,J) between nodes (I-1,J) and (I,J), I in [0,nx+1] */
    int dw = nx + 2, dh = ny + 1;
    double *fxm = dalloc((size_t)dw * dh), *fxu = dalloc((size_t)dw * dh), *fxv = dalloc((size_t)dw * dh);
#pragma omp parallel for schedule(static)
    for (int J = 0; J <= ny; ++J)
      for (int I = 0; I <= nx + 1; ++I) {
        double phi = 0.25 * (c->muX[XI(c, I - 1, J - 1)] + c->muX[XI(c, I, J - 1)] +
                             c->muX[XI(c, I - 1, J)] + c->muX[XI(c, I, J)]);
        int D = phi > 0.0 ? I - 1 : I;
        double sg = phi > 0.0 ? 1.0 : -1.0;
        int pD = NI(c, D, J);
        double vu = c->uLx[pD], vv = c->uLy[pD];
        if (order >= 2) {
          double df = 0.5 * (c->dpx[NI(c, I - 1, J)] + c->dpx[NI(c, I, J)]);
          double off = 0.5 * (sg * dual_wx(c, D, J) - df);
          vu += dual_slope(c, c->uLx, D, J, 1, 0, 1.0, 0.0) * off;
          vv += dual_slope(c, c->uLy, D, J, 1, 0, 1.0, 0.0) * off;
        }
        fxm[J * dw + I] = phi;
        fxu[J * dw + I] = phi * vu;
        fxv[J * dw + I] = phi * vv;
      }
    /* dual y-face (I,J) between nodes (I,J-1) and (I,J), J in [0,ny+1] */
    int ew = nx + 1, eh = ny + 2;
    double *fym = dalloc((size_t)ew * eh), *fyu = dalloc((size_t)ew * eh), *fyv = dalloc((size_t)ew * eh);
#pragma omp parallel for schedule(static)
    for (int J = 0; J <= ny + 1; ++J)
      for (int I = 0; I <= nx; ++I) {
        double phi = 0.25 * (c->muY[YI(c, I - 1, J - 1)] + c->muY[YI(c, I, J - 1)] +
                             c->muY[YI(c, I - 1, J)] + c->muY[YI(c, I, J)]);
        int D = phi > 0.0 ? J - 1 : J;
        double sg = phi > 0.0 ? 1.0 : -1.0;
        int pD = NI(c, I, D);
        double vu = c->uLx[pD], vv = c->uLy[pD];
        if (order >= 2) {
          double df = 0.5 * (c->dpy[NI(c, I, J - 1)] + c->dpy[NI(c, I, J)]);
          double off = 0.5 * (sg * dual_wy(c, I, D) - df);
          vu += dual_slope(c, c->uLx, I, D, 0, 1, 0.0, 1.0) * off;
          vv += dual_slope(c, c->uLy, I, D, 0, 1, 0.0, 1.0) * off;
        }
        fym[J * ew + I] = phi;
        fyu[J * ew + I] = phi * vu;
        fyv[J * ew + I] = phi * vv;
      }
    /* dual corners at cell centres (i,j), i in [-1,nx], j in [-1,ny]:
     * main diagonal between nodes (i,j) and (i+1,j+1), anti between (i,j+1)
     * and (i+1,j); each the mean of the four same-kind corner fluxes */
    int gw = nx + 2, gh = ny + 2;
    double *cdm = dalloc((size_t)gw * gh), *cdu = dalloc((size_t)gw * gh), *cdv = dalloc((size_t)gw * gh);
    double *cam = dalloc((size_t)gw * gh), *cau = dalloc((size_t)gw * gh), *cav = dalloc((size_t)gw * gh);
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= ny; ++j)
      for (int i = -1; i <= nx; ++i) {
        int h = (j + 1) * gw + (i + 1);
        double dcx = 0.25 * (c->dpx[NI(c, i, j)] + c->dpx[NI(c, i + 1, j)] +
                             c->dpx[NI(c, i, j + 1)] + c->dpx[NI(c, i + 1, j + 1)]);
        double dcy = 0.25 * (c->dpy[NI(c, i, j)] + c->dpy[NI(c, i + 1, j)] +
                             c->dpy[NI(c, i, j + 1)] + c->dpy[NI(c, i + 1, j + 1)]);
        /* main diagonal */
        double phi = 0.25 * (c->muD[NI(c, i, j)] + c->muD[NI(c, i + 1, j)] +
                             c->muD[NI(c, i, j + 1)] + c->muD[NI(c, i + 1, j + 1)]);
        int DI = phi > 0.0 ? i : i + 1, DJ = phi > 0.0 ? j : j + 1;
        double sg = phi > 0.0 ? 1.0 : -1.0;
        double vu = c->uLx[NI(c, DI, DJ)], vv = c->uLy[NI(c, DI, DJ)];
        if (order >= 2) {
          double vx = c->dx / nrm, vy = c->dy / nrm;
          double off = 0.5 * ((sg * dual_wx(c, DI, DJ) - dcx) * vx + (sg * dual_wy(c, DI, DJ) - dcy) * vy);
          vu += dual_slope(c, c->uLx, DI, DJ, 1, 1, vx, vy) * off;
          vv += dual_slope(c, c->uLy, DI, DJ, 1, 1, vx, vy) * off;
        }
        cdm[h] = phi; cdu[h] = phi * vu; cdv[h] = phi * vv;
        /* anti-diagonal: positive from top-left to bottom-right */
        phi = 0.25 * (c->muA[NI(c, i, j)] + c->muA[NI(c, i + 1, j)] +
                      c->muA[NI(c, i, j + 1)] + c->muA[NI(c, i + 1, j + 1)]);
        DI = phi > 0.0 ? i : i + 1;
        DJ = phi > 0.0 ? j + 1 : j;
        sg = phi > 0.0 ? 1.0 : -1.0;
        vu = c->uLx[NI(c, DI, DJ)];
        vv = c->uLy[NI(c, DI, DJ)];
        if (order >= 2) {
          double vx = c->dx / nrm, vy = -c->dy / nrm;
          double off = 0.5 * ((sg * dual_wx(c, DI, DJ) - dcx) * vx + (-sg * dual_wy(c, DI, DJ) - dcy) * vy);
          vu += dual_slope(c, c->uLx, DI, DJ, 1, -1, vx, vy) * off;
          vv += dual_slope(c, c->uLy, DI, DJ, 1, -1, vx, vy) * off;
        }
        cam[h] = phi; cau[h] = phi * vu; cav[h] = phi * vv;
      }
    /* nodal momentum update, order W, E, S, N, SW, NE, NW, SE */
    int badm = 0;
#pragma omp parallel for schedule(static) reduction(| : badm)
    for (int J = 0; J <= ny; ++J)
      for (int I = 0; I <= nx; ++I) {
        int p = NI(c, I, J);
        int hW = J * dw + I, hE = J * dw + I + 1;
        int hS = J * ew + I, hN = (J + 1) * ew + I;
        int hSW = J * gw + I, hNE = (J + 1) * gw + I + 1; /* cells (I-1,J-1), (I,J) */
        int hNW = (J + 1) * gw + I, hSE = J * gw + I + 1; /* cells (I-1,J), (I,J-1) */
        double m = c->mp[p];
        double mu = c->mp[p] * c->uLx[p], mv = c->mp[p] * c->uLy[p];
        m += fxm[hW]; mu += fxu[hW]; mv += fxv[hW];
        m -= fxm[hE]; mu -= fxu[hE]; mv -= fxv[hE];
        m += fym[hS]; mu += fyu[hS]; mv += fyv[hS];
        m -= fym[hN]; mu -= fyu[hN]; mv -= fyv[hN];
        m += cdm[hSW]; mu += cdu[hSW]; mv += cdv[hSW];
        m -= cdm[hNE]; mu -= cdu[hNE]; mv -= cdv[hNE];
        m += cam[hNW]; mu += cau[hNW]; mv += cav[hNW];
        m -= cam[hSE]; mu -= cau[hSE]; mv -= cav[hSE];
        if (!(m > 0.0)) badm = 1;
        c->ux[p] = mu / m;
        c->uy[p] = mv / m;
      }
    if (badm) rc = fail(c, LR_REF_ENEGATIVE, "nodal mass <= 0 after remap");
    wall_nodes(c, c->ux, c->uy);
    free(fxm); free(fxu); free(fxv); free(fym); free(fyu); free(fyv);
    free(cdm); free(cdu); free(cdv); free(cam); free(cau); free(cav);
  }

  return rc;
}

/* ------------------------------------------------------------------------ */
/* Alternate-direction (AD) remap, the paper's comparator (§2.1.1, §2.1.2,
 * §4.2): an X pass over the x-faces only, then a Y pass over the y-faces only
 * (Y then X on every second step, §2.1.2 remark 3), each a one-dimensional
 * remap of the cell and nodal quantities with its own interface. */

/* §2.1.1: x-face (I,j) flux of the X pass: the rectangle of full cell height
 * and width w = dt u_f, u_f the mean x-velocity of the face's two nodes */
static void ad_xface_region(const lr_ref_ctx *c, int I, int j, region *r) {
  memset(r, 0, sizeof *r);
  double w = 0.5 * (c->dpx[NI(c, I, j)] + c->dpx[NI(c, I, j + 1)]);
  r->type = 0; r->I = I; r->J = j;
  r->vol = fabs(w * c->dy);
  if (w >= 0.0) { r->di = I - 1; r->dj = j; r->ri = I; r->rj = j; r->sgn = 1; }
  else { r->di = I; r->dj = j; r->ri = I - 1; r->rj = j; r->sgn = -1; }
  r->rx0 = fmin(0.0, w); r->rx1 = fmax(0.0, w);
  r->ry0 = 0.0; r->ry1 = c->dy;
}

/* §2.1.2: y-face (i,J) flux of the Y pass, x and y exchanged */
static void ad_yface_region(const lr_ref_ctx *c, int i, int J, region *r) {
  memset(r, 0, sizeof *r);
  double w = 0.5 * (c->dpy[NI(c, i, J)] + c->dpy[NI(c, i + 1, J)]);
  r->type = 1; r->I = i; r->J = J;
  r->vol = fabs(w * c->dx);
  if (w >= 0.0) { r->di = i; r->dj = J - 1; r->ri = i; r->rj = J; r->sgn = 1; }
  else { r->di = i; r->dj = J; r->ri = i; r->rj = J - 1; r->sgn = -1; }
  r->rx0 = 0.0; r->rx1 = c->dx;
  r->ry0 = fmin(0.0, w); r->ry1 = fmax(0.0, w);
}

/* One pass along x (dir 0) or y (dir 1).  Its input is the state (V, M, E)
 * and the nodal velocity (ux, uy) left by the previous pass (the Lagrangian
 * state for the first pass: e = e^lag, u = u^lag); it leaves the projected
 * state in the same arrays. */
static int ad_pass(lr_ref_ctx *c, int dir, int first) {
  int C = ncell(c), nm = c->nmat, nx = c->nx, ny = c->ny;
  int rc = LR_REF_OK;
  for (int a = 0; a < nm; ++a) {
    ghost_cells(c, c->V + a * C);
    ghost_cells(c, c->M + a * C);
    ghost_cells(c, c->E + a * C);
  }
  /* §4.2: the pass starts from the volume fractions, specific energies and
   * nodal masses of its input state (k^{lagy} = k^{projx}, e^{lagy} = e^{projx}) */
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int q = CI(c, i, j);
      double Msum = 0.0;
      for (int a = 0; a < nm; ++a) {
        int qa = a * C + q;
        c->k[qa] = c->V[qa] / c->A;
        if (!first) c->eL[qa] = c->M[qa] > 0.0 ? c->E[qa] / c->M[qa] : 0.0;
        Msum += c->M[qa];
      }
      c->Mc[q] = Msum;
    }
  for (int a = 0; a < nm; ++a) ghost_cells(c, c->k + a * C);
  ghost_cells(c, c->Mc);
  nodal_mass(c);
  ghost_nodes_scalar(c, c->mp);
  ghost_nodes_vec(c, c->ux, c->uy);

  /* regions of this direction */
  int nreg = dir == 0 ? (nx + 1) * ny : nx * (ny + 1);
  region *reg = (region *)calloc((size_t)nreg, sizeof(region));
  if (!reg) return fail(c, LR_REF_ENOMEM, "out of memory");
#define ADR(i, j) (dir == 0 ? &reg[(j) * (nx + 1) + (i)] : &reg[(j) * nx + (i)])
  if (dir == 0) {
    for (int j = 0; j < ny; ++j)
      for (int I = 0; I <= nx; ++I) ad_xface_region(c, I, j, ADR(I, j));
  } else {
    for (int J = 0; J <= ny; ++J)
      for (int i = 0; i < nx; ++i) ad_yface_region(c, i, J, ADR(i, J));
  }
  /* the two regions of cell (i,j): W, E (X pass) or S, N (Y pass) */
#define AD_CELL_REGIONS(rs, i, j)                                  \
  do {                                                             \
    if (dir == 0) { rs[0] = ADR(i, j); rs[1] = ADR((i) + 1, j); }  \
    else { rs[0] = ADR(i, j); rs[1] = ADR(i, (j) + 1); }           \
  } while (0)

  /* the pass's Lagrangian volume (reading R1: A + outflow - inflow),
   * centre and width along dir, density rho^{lagx} = m / (k Vol^{lagx}) */
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int q = CI(c, i, j);
      region *rs[2];
      AD_CELL_REGIONS(rs, i, j);
      double v = c->A;
      for (int s = 0; s < 2; ++s) {
        if (is_donor(rs[s], i, j)) v += rs[s]->vol;
        else if (is_receiver(rs[s], i, j)) v -= rs[s]->vol;
      }
      c->volcf[q] = v;
      if (!(v > 0.0)) rc = fail(c, LR_REF_ENEGATIVE, "Lagrangian volume of a pass <= 0");
      int bl = NI(c, i, j), br = NI(c, i + 1, j), tl = NI(c, i, j + 1), tr = NI(c, i + 1, j + 1);
      c->xcL[q] = dir == 0 ? 0.25 * (c->xLx[bl] + c->xLx[br] + c->xLx[tl] + c->xLx[tr])
                           : c->o.x0 + (i + 0.5) * c->dx;
      c->ycL[q] = dir == 1 ? 0.25 * (c->xLy[bl] + c->xLy[br] + c->xLy[tl] + c->xLy[tr])
                           : c->o.y0 + (j + 0.5) * c->dy;
      c->dxL[q] = dir == 0 ? c->dx + 0.5 * ((c->dpx[br] + c->dpx[tr]) - (c->dpx[bl] + c->dpx[tl]))
                           : c->dx;
      c->dyL[q] = dir == 1 ? c->dy + 0.5 * ((c->dpy[tl] + c->dpy[tr]) - (c->dpy[bl] + c->dpy[br]))
                           : c->dy;
      int np = 0, m = -1;
      for (int a = 0; a < nm; ++a) {
        int qa = a * C + q;
        if (present(c, c->V[qa])) { ++np; m = a; }
        c->rhocf[qa] = present(c, c->V[qa]) ? c->M[qa] / (c->k[qa] * v) : 0.0;
      }
      c->pure[q] = np == 1 ? m : -1;
    }
  for (int a = 0; a < nm; ++a) {
    ghost_cells(c, c->rhocf + a * C);
    ghost_cells(c, c->eL + a * C);
  }
  ghost_cells(c, c->volcf);
  ghost_cells_coord(c, c->xcL, 0);
  ghost_cells_coord(c, c->ycL, 1);
  ghost_cells(c, c->dxL);
  ghost_cells(c, c->dyL);
  ghost_cells_int(c, c->pure);

  /* §4.2: partial volumes from the interface placed on the pass's Lagrangian
   * cell (only its faces along dir move), reconstruction, update */
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      region *rs[2];
      AD_CELL_REGIONS(rs, i, j);
      donor_partials(c, rs, 2, i, j, dir == 0, dir == 1, c->volcf[CI(c, i, j)]);
    }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      region *rs[2];
      AD_CELL_REGIONS(rs, i, j);
      donor_fluxes(c, rs, 2, i, j);
    }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      region *rs[2];
      AD_CELL_REGIONS(rs, i, j);
      primal_update(c, rs, 2, i, j, c->volcf[CI(c, i, j)]);
    }

  /* signed total mass fluxes of the pass's faces, mirrored at the walls */
  if (dir == 0) {
    for (int p = 0; p < nxf(c); ++p) c->muX[p] = 0.0;
    for (int j = 0; j < ny; ++j)
      for (int I = 0; I <= nx; ++I) {
        region *r = ADR(I, j);
        double m = 0.0;
        for (int a = 0; a < nm; ++a) m += r->mu[a];
        c->muX[XI(c, I, j)] = r->sgn * m;
      }
    for (int j = -G; j < ny + G; ++j)
      for (int I = -G; I <= nx + G; ++I) {
        int rI = mn(I, nx), rj = mc(j, ny);
        if (rI == I && rj == j) continue;
        c->muX[XI(c, I, j)] = (rI != I ? -1.0 : 1.0) * c->muX[XI(c, rI, rj)];
      }
  } else {
    for (int p = 0; p < nyf(c); ++p) c->muY[p] = 0.0;
    for (int J = 0; J <= ny; ++J)
      for (int i = 0; i < nx; ++i) {
        region *r = ADR(i, J);
        double m = 0.0;
        for (int a = 0; a < nm; ++a) m += r->mu[a];
        c->muY[YI(c, i, J)] = r->sgn * m;
      }
    for (int J = -G; J <= ny + G; ++J)
      for (int i = -G; i < nx + G; ++i) {
        int ri = mc(i, nx), rJ = mn(J, ny);
        if (ri == i && rJ == J) continue;
        c->muY[YI(c, i, J)] = (rJ != J ? -1.0 : 1.0) * c->muY[YI(c, ri, rJ)];
      }
  }
  free(reg);
#undef AD_CELL_REGIONS
#undef ADR

  /* §2.1.1 dual mesh: nodal momentum through the two dual faces along dir,
   * each carrying 1/4 of the four same-side primal face mass fluxes; the
   * velocity reconstructed as on the primal mesh (dual centres at the
   * Lagrangian node positions, reading) */
  if (!c->o.kinematic) {
    int order = c->o.recon_order;
    int nf = dir == 0 ? (nx + 2) * (ny + 1) : (nx + 1) * (ny + 2);
    double *fm = dalloc(nf), *fu = dalloc(nf), *fv = dalloc(nf);
    double *nu = dalloc((size_t)(nx + 1) * (ny + 1)), *nv = dalloc((size_t)(nx + 1) * (ny + 1));
    if (!fm || !fu || !fv || !nu || !nv) {
      free(fm); free(fu); free(fv); free(nu); free(nv);
      return fail(c, LR_REF_ENOMEM, "out of memory");
    }
    if (dir == 0) {
      /* dual x-face (I,J) between nodes (I-1,J) and (I,J), I in [0,nx+1] */
      for (int J = 0; J <= ny; ++J)
        for (int I = 0; I <= nx + 1; ++I) {
          double phi = 0.25 * (c->muX[XI(c, I - 1, J - 1)] + c->muX[XI(c, I, J - 1)] +
                               c->muX[XI(c, I - 1, J)] + c->muX[XI(c, I, J)]);
          int D = phi > 0.0 ? I - 1 : I;
          double sg = phi > 0.0 ? 1.0 : -1.0;
          int pD = NI(c, D, J);
          double vu = c->ux[pD], vv = c->uy[pD];
          if (order == 2) {
            double df = 0.5 * (c->dpx[NI(c, I - 1, J)] + c->dpx[NI(c, I, J)]);
            double off = 0.5 * (sg * dual_wx(c, D, J) - df);
            vu += dual_slope(c, c->ux, D, J, 1, 0, 1.0, 0.0) * off;
            vv += dual_slope(c, c->uy, D, J, 1, 0, 1.0, 0.0) * off;
          }
          int h = J * (nx + 2) + I;
          fm[h] = phi; fu[h] = phi * vu; fv[h] = phi * vv;
        }
    } else {
      /* dual y-face (I,J) between nodes (I,J-1) and (I,J), J in [0,ny+1] */
      for (int J = 0; J <= ny + 1; ++J)
        for (int I = 0; I <= nx; ++I) {
          double phi = 0.25 * (c->muY[YI(c, I - 1, J - 1)] + c->muY[YI(c, I, J - 1)] +
                               c->muY[YI(c, I - 1, J)] + c->muY[YI(c, I, J)]);
          int D = phi > 0.0 ? J - 1 : J;
          double sg = phi > 0.0 ? 1.0 : -1.0;
          int pD = NI(c, I, D);
          double vu = c->ux[pD], vv = c->uy[pD];
          if (order == 2) {
            double df = 0.5 * (c->dpy[NI(c, I, J - 1)] + c->dpy[NI(c, I, J)]);
            double off = 0.5 * (sg * dual_wy(c, I, D) - df);
            vu += dual_slope(c, c->ux, I, D, 0, 1, 0.0, 1.0) * off;
            vv += dual_slope(c, c->uy, I, D, 0, 1, 0.0, 1.0) * off;
          }
          int h = J * (nx + 1) + I;
          fm[h] = phi; fu[h] = phi * vu; fv[h] = phi * vv;
        }
    }
    /* m_p^{proj} u^{proj} = m_p u + in - out through the low then high face */
    for (int J = 0; J <= ny; ++J)
      for (int I = 0; I <= nx; ++I) {
        int p = NI(c, I, J);
        int lo = dir == 0 ? J * (nx + 2) + I : J * (nx + 1) + I;
        int hi = dir == 0 ? lo + 1 : lo + (nx + 1);
        double m = c->mp[p];
        double mu = c->mp[p] * c->ux[p], mv = c->mp[p] * c->uy[p];
        m += fm[lo]; mu += fu[lo]; mv += fv[lo];
        m -= fm[hi]; mu -= fu[hi]; mv -= fv[hi];
        if (!(m > 0.0)) rc = fail(c, LR_REF_ENEGATIVE, "nodal mass <= 0 after a pass");
        nu[J * (nx + 1) + I] = mu / m;
        nv[J * (nx + 1) + I] = mv / m;
      }
    for (int J = 0; J <= ny; ++J)
      for (int I = 0; I <= nx; ++I) {
        c->ux[NI(c, I, J)] = nu[J * (nx + 1) + I];
        c->uy[NI(c, I, J)] = nv[J * (nx + 1) + I];
      }
    wall_nodes(c, c->ux, c->uy);
    free(fm); free(fu); free(fv); free(nu); free(nv);
  }
  return rc;
}

/* the whole AD remap: X then Y on the first, third, ... step of a run and Y
 * then X on the others (§2.1.2 remark 3) */
static int remap_ad(lr_ref_ctx *c) {
  int N = nnode(c);
  /* the passes carry the nodal velocity from u^lag on */
  for (int p = 0; p < N; ++p) { c->ux[p] = c->uLx[p]; c->uy[p] = c->uLy[p]; }
  int xfirst = (c->step % 2) == 0;
  int rc1 = ad_pass(c, xfirst ? 0 : 1, 1);
  if (rc1 == LR_REF_ENOMEM) return rc1;
  int rc2 = ad_pass(c, xfirst ? 1 : 0, 0);
  if (rc2 == LR_REF_ENOMEM) return rc2;
  return rc2 != LR_REF_OK ? rc2 : rc1;
}

/* ------------------------------------------------------------------------ */
static int step_once(lr_ref_ctx *c, double t_end, double *dt_out, int *last) {
  int C = ncell(c), N = nnode(c), nm = c->nmat, nx = c->nx, ny = c->ny;
  *last = 0;
  memset(c->flags, 0, (size_t)C * sizeof(int));
  for (int a = 0; a < nm; ++a) {
    ghost_cells(c, c->V + a * C);
    ghost_cells(c, c->M + a * C);
    ghost_cells(c, c->E + a * C);
  }
  ghost_nodes_vec(c, c->ux, c->uy);
  derived(c);

  /* time step */
  double dt = c->o.fixed_dt > 0.0 ? c->o.fixed_dt : cfl_dt(c);
  if (t_end - c->t <= dt) { dt = t_end - c->t; *last = 1; }
  if (!(dt > 0.0) || !isfinite(dt)) return fail(c, LR_REF_EDT, "time step underflow or not finite");
  c->last_dt = dt;

  /* Lagrangian phase */
  if (c->o.kinematic) {
    for (int q = 0; q < C; ++q) c->Q[q] = 0.0;
    nodal_mass(c);
    kinematic_lagrange(c, dt);
  } else {
    pseudo_viscosity(c);
    nodal_mass(c);
    predictor(c, dt);
    corrector(c, dt);
  }
  for (int p = 0; p < N; ++p) { c->xLx[p] = 0; c->xLy[p] = 0; }
  for (int J = 0; J <= ny; ++J)
    for (int I = 0; I <= nx; ++I) {
      int p = NI(c, I, J);
      c->xLx[p] = node_x(c, I) + c->dpx[p];
      c->xLy[p] = node_y(c, J) + c->dpy[p];
    }
  ghost_nodes_vec(c, c->dpx, c->dpy);
  ghost_nodes_vec(c, c->uhx, c->uhy);
  ghost_nodes_vec(c, c->uLx, c->uLy);
  ghost_nodes_pos(c, c->xLx, c->xLy);
  ghost_nodes_scalar(c, c->mp);

  int rc = c->o.remap == LR_REF_REMAP_AD ? remap_ad(c) : remap_directcf(c);
  if (rc == LR_REF_ENOMEM) return rc;

  /* finish */
  c->t = *last ? t_end : c->t + dt;
  c->step += 1;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i)
      for (int b = 0; b < LR_REF_NCOUNT; ++b)
        if (c->flags[CI(c, i, j)] & (1 << b)) c->counts[b] += 1;
  *dt_out = dt;
  /* a partial quantity below -1e-10 of the cell's total counts as negative;
   * smaller negatives are the rounding left by a material that moved out */
  for (int j = 0; j < ny && rc == LR_REF_OK; ++j)
    for (int i = 0; i < nx && rc == LR_REF_OK; ++i) {
      double Ms = 0.0, Es = 0.0;
      for (int a = 0; a < nm; ++a) {
        Ms += fabs(c->M[a * C + CI(c, i, j)]);
        Es += fabs(c->E[a * C + CI(c, i, j)]);
      }
      for (int a = 0; a < nm; ++a) {
        int qa = a * C + CI(c, i, j);
        double V = c->V[qa], M = c->M[qa], E = c->E[qa];
        if (!isfinite(V) || !isfinite(M) || !isfinite(E)) { rc = fail(c, LR_REF_ENAN, "NaN in state"); break; }
        if (V < -1e-10 * c->A || M < -1e-10 * Ms || E < -1e-10 * Es) {
          rc = fail(c, LR_REF_ENEGATIVE, "negative partial volume, mass or energy");
          break;
        }
      }
    }
  for (int J = 0; J <= ny && rc == LR_REF_OK; ++J)
    for (int I = 0; I <= nx; ++I)
      if (!isfinite(c->ux[NI(c, I, J)]) || !isfinite(c->uy[NI(c, I, J)])) {
        rc = fail(c, LR_REF_ENAN, "NaN in velocity");
        break;
      }
  return rc;
}

int lr_ref_step(lr_ref_ctx *c, double *dt_out) {
  if (!c) return LR_REF_EINVAL;
  if (!c->have_state) return fail(c, LR_REF_ESTATE, "no state set");
  double dt = 0.0;
  int last = 0;
  int rc = step_once(c, INFINITY, &dt, &last);
  if (dt_out) *dt_out = dt;
  return rc;
}

int lr_ref_run(lr_ref_ctx *c, double t_end, long max_steps, long *steps_out, double *t_out) {
  if (!c) return LR_REF_EINVAL;
  if (!c->have_state) return fail(c, LR_REF_ESTATE, "no state set");
  if (!(t_end >= c->t) || max_steps < 0) return fail(c, LR_REF_EINVAL, "t_end < t or max_steps < 0");
  long n = 0;
  int rc = LR_REF_OK;
  while (n < max_steps && c->t < t_end) {
    double dt;
    int last;
    rc = step_once(c, t_end, &dt, &last);
    ++n;
    if (rc != LR_REF_OK || last) break;
  }
  if (steps_out) *steps_out = n;
  if (t_out) *t_out = c->t;
  return rc;
}

/* ------------------------------------------------------------------------ */
/* outputs                                                                   */
int lr_ref_get_fields(lr_ref_ctx *c, unsigned mask, double *const *out) {
  if (!c || !out) return LR_REF_EINVAL;
  if (!c->have_state) return fail(c, LR_REF_ESTATE, "no state set");
  int nx = c->nx, ny = c->ny, nm = c->nmat, C = ncell(c);
  size_t cells = (size_t)nx * ny;
  int slot = 0;
  for (unsigned bit = 1; bit <= LR_REF_F_IE; bit <<= 1) {
    if (!(mask & bit)) continue;
    double *o = out[slot++];
    if (!o) return LR_REF_EINVAL;
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int q = CI(c, i, j);
        size_t h = (size_t)j * nx + i;
        double Ms = 0, Es = 0, Ps = 0;
        for (int a = 0; a < nm; ++a) {
          int qa = a * C + q;
          double V = c->V[qa], M = c->M[qa], E = c->E[qa];
          int pr = present(c, V);
          double rho = pr ? M / V : 0.0, e = (pr && M > 0) ? E / M : 0.0;
          double P = pr ? eos_p(c, a, rho, e) : 0.0;
          Ms += M; Es += E; Ps += (V / c->A) * P;
          switch (bit) {
            case LR_REF_F_K: o[a * cells + h] = V / c->A; break;
            case LR_REF_F_RHOA: o[a * cells + h] = rho; break;
            case LR_REF_F_EA: o[a * cells + h] = e; break;
            case LR_REF_F_PA: o[a * cells + h] = P; break;
            case LR_REF_F_VOL: o[a * cells + h] = V; break;
            case LR_REF_F_MASS: o[a * cells + h] = M; break;
            case LR_REF_F_IE: o[a * cells + h] = E; break;
            default: break;
          }
        }
        if (bit == LR_REF_F_RHO) o[h] = Ms / c->A;
        if (bit == LR_REF_F_P) o[h] = Ps;
        if (bit == LR_REF_F_E) o[h] = Ms > 0 ? Es / Ms : 0.0;
      }
    if (bit == LR_REF_F_UX || bit == LR_REF_F_UY)
      for (int J = 0; J <= ny; ++J)
        for (int I = 0; I <= nx; ++I)
          o[(size_t)J * (nx + 1) + I] = bit == LR_REF_F_UX ? c->ux[NI(c, I, J)] : c->uy[NI(c, I, J)];
  }
  return LR_REF_OK;
}

int lr_ref_totals(lr_ref_ctx *c, double *out) {
  if (!c || !out) return LR_REF_EINVAL;
  if (!c->have_state) return fail(c, LR_REF_ESTATE, "no state set");
  int nx = c->nx, ny = c->ny, nm = c->nmat, C = ncell(c);
  double Et = 0.0;
  for (int a = 0; a < nm; ++a) {
    double sv = 0, sm = 0, se = 0;
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int qa = a * C + CI(c, i, j);
        sv += c->V[qa]; sm += c->M[qa]; se += c->E[qa];
      }
    out[a] = sv; out[nm + a] = sm; out[2 * nm + a] = se;
    Et += se;
  }
  double px = 0, py = 0;
  for (int J = 0; J <= ny; ++J)
    for (int I = 0; I <= nx; ++I) {
      double m = 0.0;
      for (int b = -1; b <= 0; ++b)
        for (int a = -1; a <= 0; ++a) {
          int i = I + a, j = J + b;
          if (i < 0 || j < 0 || i >= nx || j >= ny) continue;
          for (int s = 0; s < nm; ++s) m += 0.25 * c->M[s * C + CI(c, i, j)];
        }
      double u = c->ux[NI(c, I, J)], v = c->uy[NI(c, I, J)];
      px += m * u; py += m * v;
      Et += 0.5 * m * (u * u + v * v);
    }
  out[3 * nm] = px; out[3 * nm + 1] = py; out[3 * nm + 2] = Et;
  return LR_REF_OK;
}

/* stage arrays (cells [nx*ny], per-material [nmat][nx*ny], nodes [(nx+1)(ny+1)],
 * x-faces [ny][nx+1], y-faces [ny+1][nx], per-material faces [nmat][...]) */
int lr_ref_debug_get(lr_ref_ctx *c, const char *name, double *out) {
  if (!c || !name || !out) return LR_REF_EINVAL;
  int nx = c->nx, ny = c->ny, nm = c->nmat, C = ncell(c), N = nnode(c);
  size_t cells = (size_t)nx * ny;
  struct { const char *n; double *a; int per_mat; } cellf[] = {
      {"Q", c->Q, 0}, {"Pc", c->Pc, 0}, {"cc", c->cc, 0}, {"S", c->S, 0},
      {"VL", c->VL, 0}, {"volcf", c->volcf, 0}, {"xcL", c->xcL, 0}, {"ycL", c->ycL, 0},
      {"dxL", c->dxL, 0}, {"dyL", c->dyL, 0}, {"eL", c->eL, 1}, {"rhocf", c->rhocf, 1},
      {"P_half", c->P_half, 1}, {"e_half", c->e_half, 1}};
  for (size_t s = 0; s < sizeof cellf / sizeof cellf[0]; ++s) {
    if (strcmp(name, cellf[s].n)) continue;
    int nmm = cellf[s].per_mat ? nm : 1;
    for (int a = 0; a < nmm; ++a)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) out[a * cells + (size_t)j * nx + i] = cellf[s].a[a * C + CI(c, i, j)];
    return LR_REF_OK;
  }
  struct { const char *n; double *a; } nodef[] = {
      {"mp", c->mp}, {"uhx", c->uhx}, {"uhy", c->uhy}, {"uLx", c->uLx}, {"uLy", c->uLy},
      {"dpx", c->dpx}, {"dpy", c->dpy}, {"muD", c->muD}, {"muA", c->muA}, {"Wc", c->Wc}};
  for (size_t s = 0; s < sizeof nodef / sizeof nodef[0]; ++s) {
    if (strcmp(name, nodef[s].n)) continue;
    for (int J = 0; J <= ny; ++J)
      for (int I = 0; I <= nx; ++I) out[(size_t)J * (nx + 1) + I] = nodef[s].a[NI(c, I, J)];
    return LR_REF_OK;
  }
  if (!strcmp(name, "Wpc")) {
    for (int a = 0; a < nm; ++a)
      for (int J = 0; J <= ny; ++J)
        for (int I = 0; I <= nx; ++I)
          out[a * (size_t)(nx + 1) * (ny + 1) + (size_t)J * (nx + 1) + I] = c->Wpc[a * N + NI(c, I, J)];
    return LR_REF_OK;
  }
  if (!strcmp(name, "muX") || !strcmp(name, "Wx")) {
    double *a = name[0] == 'm' ? c->muX : c->Wx;
    for (int j = 0; j < ny; ++j)
      for (int I = 0; I <= nx; ++I) out[(size_t)j * (nx + 1) + I] = a[XI(c, I, j)];
    return LR_REF_OK;
  }
  if (!strcmp(name, "Wpx")) {
    for (int s = 0; s < nm; ++s)
      for (int j = 0; j < ny; ++j)
        for (int I = 0; I <= nx; ++I)
          out[s * (size_t)(nx + 1) * ny + (size_t)j * (nx + 1) + I] = c->Wpx[s * nxf(c) + XI(c, I, j)];
    return LR_REF_OK;
  }
  if (!strcmp(name, "muY") || !strcmp(name, "Wy")) {
    double *a = name[0] == 'm' ? c->muY : c->Wy;
    for (int J = 0; J <= ny; ++J)
      for (int i = 0; i < nx; ++i) out[(size_t)J * nx + i] = a[YI(c, i, J)];
    return LR_REF_OK;
  }
  if (!strcmp(name, "Wpy")) {
    for (int s = 0; s < nm; ++s)
      for (int J = 0; J <= ny; ++J)
        for (int i = 0; i < nx; ++i)
          out[s * (size_t)nx * (ny + 1) + (size_t)J * nx + i] = c->Wpy[s * nyf(c) + YI(c, i, J)];
    return LR_REF_OK;
  }
  if (!strcmp(name, "dt")) { out[0] = c->last_dt; return LR_REF_OK; }
  if (!strcmp(name, "counts")) {
    for (int b = 0; b < LR_REF_NCOUNT; ++b) out[b] = (double)c->counts[b];
    return LR_REF_OK;
  }
  if (!strcmp(name, "t")) { out[0] = c->t; return LR_REF_OK; }
  return fail(c, LR_REF_EINVAL, "unknown stage name");
}
