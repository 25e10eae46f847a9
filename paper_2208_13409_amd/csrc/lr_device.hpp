// lr_device.hpp — device helpers of the DirectCF Lagrange–Remap kernels
// (gfx950).  Geometry of the flux volumes (paper §2.3), closed-form
// rectangle / half-plane areas and their inverse for the VOF interface (§4.4),
// the Van Leer limited slope (§2.1.1) and the wall mirrors.
#pragma once
#include <hip/hip_runtime.h>

#include "lr.h"

namespace lr {

constexpr int MAXMAT = LR_MAXMAT;

// Problem constants, passed by value to every kernel.
struct Grid {
  int nx, ny, nmat;
  int recon_order, kinematic;
  double dx, dy, A;     // cell sizes and area
  double Lx, Ly;        // domain extents x1-x0, y1-y0
  double cfl, a1, a2, k_eps, fixed_dt;
  double gamma[MAXMAT];
};

// Device-resident time-stepping control: the host never needs dt per step.
struct Scalars {
  double t;                  // time at the start of the current step
  double dt;                 // time step of the current step
  double t_end;              // end of the current run
  unsigned long long dtmin;  // bits of the next CFL bound (positive double), atomicMin target
  long long step;            // steps taken since lr_set_state
  long long step_limit;      // the run stops when step reaches it
  int last;                  // the current step lands on t_end
  int done;                  // no step is pending: kernels return at once
  int err;                   // error bits (ERR_*)
  int pad;
};

enum { ERR_NEG = 1, ERR_NAN = 2, ERR_DT = 4, ERR_VOLCF = 8, ERR_NODEMASS = 16 };

// ---------------------------------------------------------------- indexing
__device__ __forceinline__ int refl_cell(int i, int n) {
  return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i);
}
__device__ __forceinline__ int refl_node(int I, int n) {
  return I < 0 ? -I : (I > n ? 2 * n - I : I);
}

// ---------------------------------------------------------------- limiter
// Van Leer: for one-sided slopes of the same sign, the harmonic mean
// 2 dm dp / (dm + dp); otherwise 0 (the limiter of §2.1.1 written out).
__device__ __forceinline__ double van_leer(double dm, double dp) {
  return (dm * dp > 0.0) ? 2.0 * dm * dp / (dm + dp) : 0.0;
}

// ---------------------------------------------------------------- geometry
// Quadrilateral area F of §1.2 from node positions relative to a common origin:
// half the absolute cross product of the left and bottom edges plus half that
// of the right and top edges.
__device__ __forceinline__ double quad_area(double blx, double bly, double brx, double bry,
                                            double tlx, double tly, double trx, double try_) {
  const double lx = tlx - blx, ly = tly - bly;
  const double bx = brx - blx, by = bry - bly;
  const double rx = trx - brx, ry = try_ - bry;
  const double tx = trx - tlx, ty = try_ - tly;
  return 0.5 * fabs(lx * by - ly * bx) + 0.5 * fabs(rx * ty - ry * tx);
}

// DirectCF face flux volume (§2.3) of a face of length D whose end nodes are
// displaced by (da_n, da_t) at the lower end and (db_n, db_t) at the upper end
// (n: component normal to the face, t: along it).  The trapezoid between the
// Eulerian face and the Lagrangian face line, cut at t- = max(0, da_t) and
// t+ = D + min(0, db_t), is replaced by a rectangle of width w (the mean
// offset of the line at t-, t+) and height h; the flux volume is w h.
struct FaceGeo {
  double w;   // signed width: > 0 flux along +n
  double h;   // height (>= 0)
  double t0;  // start of the rectangle along the face, from the lower node
};
__device__ __forceinline__ FaceGeo face_geo(double da_n, double da_t, double db_n, double db_t,
                                            double D) {
  const double tlo = fmax(0.0, da_t);
  const double thi = D + fmin(0.0, db_t);
  double h = thi - tlo;
  if (h < 0.0) h = 0.0;
  const double slope = (db_n - da_n) / ((D + db_t) - da_t);
  const double nlo = da_n + (tlo - da_t) * slope;
  const double nhi = da_n + (thi - da_t) * slope;
  FaceGeo g;
  g.w = 0.5 * (nlo + nhi);
  g.h = h;
  g.t0 = tlo;
  return g;
}

// Area of the part of the rectangle [x0,x1] x [y0,y1] where nx x + ny y >= s,
// in closed form.  With the rectangle centred (half sizes a, b), P = |nx|,
// Q = |ny| and t = P a + Q b - s' (depth of the cut below the far corner), the
// cut-off piece is a triangle t^2/(2PQ) while the line meets two adjacent
// sides, and a trapezoid 2a(t - aP)/Q or 2b(t - bQ)/P once it meets two
// opposite sides; s' < 0 uses the complement.
__device__ __forceinline__ double corner_piece(double a, double b, double P, double Q, double t) {
  if (t <= 0.0) return 0.0;
  const bool x_first = a * P <= b * Q;  // the line leaves the x-range first
  if (x_first) {
    if (t <= 2.0 * a * P) return t * t / (2.0 * P * Q);
    return 2.0 * a * (t - a * P) / Q;
  }
  if (t <= 2.0 * b * Q) return t * t / (2.0 * P * Q);
  return 2.0 * b * (t - b * Q) / P;
}
__device__ __forceinline__ double rect_halfplane_area(double x0, double x1, double y0, double y1,
                                                      double nx, double ny, double s) {
  if (!(x1 > x0) || !(y1 > y0)) return 0.0;
  const double a = 0.5 * (x1 - x0), b = 0.5 * (y1 - y0);
  const double sc = s - (nx * (0.5 * (x0 + x1)) + ny * (0.5 * (y0 + y1)));
  const double P = fabs(nx), Q = fabs(ny);
  const double h = P * a + Q * b;
  const double full = 4.0 * a * b;
  if (sc >= h) return 0.0;
  if (sc <= -h) return (x1 - x0) * (y1 - y0);
  double area;
  if (sc >= 0.0) area = corner_piece(a, b, P, Q, h - sc);
  else area = full - corner_piece(a, b, P, Q, h + sc);
  const double whole = (x1 - x0) * (y1 - y0);
  return area < 0.0 ? 0.0 : (area > whole ? whole : area);
}

// Inverse of corner_piece for T in [0, 2ab]: the depth t giving area T.
__device__ __forceinline__ double corner_depth(double a, double b, double P, double Q, double T) {
  if (T <= 0.0) return 0.0;
  if (a * P <= b * Q) {
    const double Tt = 2.0 * a * a * P / Q;  // area where the triangle reaches x-extent
    if (T <= Tt) return sqrt(2.0 * P * Q * T);
    return T * Q / (2.0 * a) + a * P;
  }
  const double Tt = 2.0 * b * b * Q / P;
  if (T <= Tt) return sqrt(2.0 * P * Q * T);
  return T * P / (2.0 * b) + b * Q;
}

// Offset s of the line n.x = s such that the part of the rectangle where
// n.x >= s has area frac*|R| (§4.4, placement of the interface), in closed
// form from the piecewise-quadratic area; frac in [0,1], n a unit vector.
__device__ __forceinline__ double interface_offset(double x0, double x1, double y0, double y1,
                                                   double nx, double ny, double frac) {
  const double a = 0.5 * (x1 - x0), b = 0.5 * (y1 - y0);
  const double P = fabs(nx), Q = fabs(ny);
  const double h = P * a + Q * b;
  const double full = 4.0 * a * b;
  const double T = frac * full;
  double sc;
  if (T <= 0.5 * full) sc = h - corner_depth(a, b, P, Q, T);
  else sc = -(h - corner_depth(a, b, P, Q, full - T));
  return sc + (nx * (0.5 * (x0 + x1)) + ny * (0.5 * (y0 + y1)));
}

}  // namespace lr
