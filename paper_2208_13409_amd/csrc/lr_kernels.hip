// lr_kernels.hip — HIP kernels (gfx950) and C-ABI of one DirectCF
// Lagrange–Remap time step (B. Chaudet, arXiv:2208.13409):
//   k_lag_cell    predictor per cell: EOS, Wilkins Q, Vol^{n+1/2}, e_a^{n+1/2},
//                 P_a^{n+1/2} (§1.2 eq. prediction, §4.1 eq. prediction_multi)
//   k_lag_node    nodal mass, gradient of P+Q, u^{n+1/2}, u^{lag} (§1.2)
//   k_remap_cell  corrector energy e_a^{lag} (§4.1 eq. correction_multi),
//                 Vol^{lagCF}, rho^{lagCF}, Lagrangian centres and widths (§2.3)
//   k_flux        every cell as a donor: its outflow face and corner regions,
//                 VOF partial volumes (§4.4), clipping, reconstruction (§2.1.1,
//                 §3.3, §4.2); each region is written once, by its donor
//   k_update_cell primal conservative update (§2.3, §4.4) + sound speed
//   k_update_node dual momentum update (§2.1.1 dual mesh, §2.3 dual corners)
//                 + wavefront-shuffle CFL min-reduction for the next step
//   k_control     device-side time control (dt, t, t_end, step count)
// Data are structure-of-arrays, x fastest; walls are handled by mirrored
// indices, never by ghost storage.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lr.h"
#include "lr_device.hpp"

using namespace lr;

namespace {

// device pointers of one context
struct Fields {
  double *V, *M, *E;            // [nmat][C] conserved partial volume, mass, energy
  double *ux, *uy;              // [N] nodal velocity
  double *Q, *S, *Mc, *Ph;      // [C],[C],[C],[nmat][C]
  double *mp, *uhx, *uhy, *uLx, *uLy;  // [N]
  double *VL, *volcf, *xcL, *ycL, *dxL, *dyL;  // [C]
  double *rhocf, *eL;           // [nmat][C]
  int *pure;                    // [C] present material if exactly one, else -1
  double *FX, *FY, *FC;         // region fluxes [3 nmat + 1][faces or nodes]
  double *cs;                   // [C] sound speed of the updated state
  Scalars *s;
};

__device__ __forceinline__ int cidx(const Grid &g, int i, int j) { return j * g.nx + i; }
__device__ __forceinline__ int nidx(const Grid &g, int I, int J) { return J * (g.nx + 1) + I; }

__device__ __forceinline__ bool present(const Grid &g, double V) { return V > g.k_eps * g.A; }

// ------------------------------------------------------------ predictor (cell)
__global__ void k_lag_cell(Grid g, Fields f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  if (f.s->done) return;
  const double dt = f.s->dt;
  const int C = g.nx * g.ny, q = cidx(g, i, j);
  const int bl = nidx(g, i, j), br = bl + 1, tl = bl + g.nx + 1, tr = tl + 1;
  double Msum = 0.0, rc2 = 0.0;
  double rho[MAXMAT], e[MAXMAT], P[MAXMAT], k[MAXMAT];
  bool pr[MAXMAT];
  for (int a = 0; a < g.nmat; ++a) {
    const double V = f.V[a * C + q], M = f.M[a * C + q], E = f.E[a * C + q];
    k[a] = V / g.A;
    pr[a] = present(g, V);
    e[a] = M > 0.0 ? E / M : 0.0;
    rho[a] = pr[a] ? M / V : 0.0;
    P[a] = pr[a] ? (g.gamma[a] - 1.0) * rho[a] * e[a] : 0.0;
    if (pr[a]) rc2 += k[a] * g.gamma[a] * P[a];
    Msum += M;
  }
  f.Mc[q] = Msum;
  double Qc = 0.0;
  if (!g.kinematic) {
    const double rhoc = Msum / g.A;
    const double c2 = rhoc > 0.0 ? rc2 / rhoc : 0.0;
    const double cc = c2 > 0.0 ? sqrt(c2) : 0.0;
    // Wilkins pseudo-viscosity with Delta u ~ L div u (§1.2)
    const double div = (f.ux[br] + f.ux[tr] - f.ux[bl] - f.ux[tl]) / (2.0 * g.dx) +
                       (f.uy[tl] + f.uy[tr] - f.uy[bl] - f.uy[br]) / (2.0 * g.dy);
    const double L = sqrt(g.A);
    if (div < 0.0) Qc = rhoc * (g.a1 * L * cc * fabs(div) + g.a2 * L * L * div * div);
    // Vol^{n+1/2} = F(x^n + dt/2 u^n), positions relative to the BL node
    const double hdt = 0.5 * dt;
    const double Vh = quad_area(hdt * f.ux[bl], hdt * f.uy[bl], g.dx + hdt * f.ux[br],
                                hdt * f.uy[br], hdt * f.ux[tl], g.dy + hdt * f.uy[tl],
                                g.dx + hdt * f.ux[tr], g.dy + hdt * f.uy[tr]);
    double Pch = 0.0;
    for (int a = 0; a < g.nmat; ++a) {
      double Ph = 0.0;
      if (pr[a]) {
        const double rho_h = f.M[a * C + q] / (k[a] * Vh);
        const double e_h = e[a] - (P[a] + Qc) * (1.0 / rho_h - 1.0 / rho[a]);
        Ph = (g.gamma[a] - 1.0) * rho_h * e_h;
        Pch += k[a] * Ph;
      }
      f.Ph[a * C + q] = Ph;
    }
    f.S[q] = Pch + Qc;
  }
  f.Q[q] = Qc;
}

// ------------------------------------------------------------ nodal phase
__global__ void k_lag_node(Grid g, Fields f) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  if (I > g.nx || J > g.ny) return;
  if (f.s->done) return;
  const double dt = f.s->dt;
  const int p = nidx(g, I, J);
  const int iw = refl_cell(I - 1, g.nx), ie = refl_cell(I, g.nx);
  const int js = refl_cell(J - 1, g.ny), jn = refl_cell(J, g.ny);
  const int sw = cidx(g, iw, js), se = cidx(g, ie, js), nw = cidx(g, iw, jn), ne = cidx(g, ie, jn);
  f.mp[p] = 0.25 * (f.Mc[sw] + f.Mc[se] + f.Mc[nw] + f.Mc[ne]);
  double uhx, uhy, uLx, uLy;
  if (g.kinematic) {
    uhx = uLx = f.ux[p];
    uhy = uLy = f.uy[p];
  } else {
    const double gx = ((f.S[se] + f.S[ne]) - (f.S[sw] + f.S[nw])) / (2.0 * g.dx);
    const double gy = ((f.S[nw] + f.S[ne]) - (f.S[sw] + f.S[se])) / (2.0 * g.dy);
    const double rho_p = f.mp[p] / g.A;
    uhx = f.ux[p] - 0.5 * dt * gx / rho_p;
    uhy = f.uy[p] - 0.5 * dt * gy / rho_p;
    if (I == 0 || I == g.nx) uhx = 0.0;
    if (J == 0 || J == g.ny) uhy = 0.0;
    uLx = 2.0 * uhx - f.ux[p];
    uLy = 2.0 * uhy - f.uy[p];
    if (I == 0 || I == g.nx) uLx = 0.0;
    if (J == 0 || J == g.ny) uLy = 0.0;
  }
  f.uhx[p] = uhx;
  f.uhy[p] = uhy;
  f.uLx[p] = uLx;
  f.uLy[p] = uLy;
}

// ------------------------------------------------------------ region geometry
// The eight flux regions touching cell (i,j): W, E, S, N faces, then the
// corners at its BL, BR, TL, TR nodes.  For each: the volume |W|, whether
// the cell is the donor (+1), the receiver (-1) or neither (0).
struct NodeD {
  double x, y;  // displacement dt u^{n+1/2}
};
__device__ __forceinline__ NodeD node_d(const Fields &f, int p, double dt) {
  NodeD d;
  d.x = dt * f.uhx[p];
  d.y = dt * f.uhy[p];
  return d;
}
// corner kind at a node: main diagonal when both displacement signs agree
__device__ __forceinline__ bool corner_main(NodeD d) { return (d.x >= 0.0) == (d.y >= 0.0); }

struct CellRegions {
  double vol[8];
  int role[8];  // +1 donor, -1 receiver, 0 not involved
  FaceGeo fg[4];
};
__device__ __forceinline__ void cell_regions(const Grid &g, NodeD bl, NodeD br, NodeD tl, NodeD tr,
                                             CellRegions &r) {
  // x-faces: normal x, tangent y; lower node first
  r.fg[0] = face_geo(bl.x, bl.y, tl.x, tl.y, g.dy);  // W face (x-face i)
  r.fg[1] = face_geo(br.x, br.y, tr.x, tr.y, g.dy);  // E face (x-face i+1)
  // y-faces: normal y, tangent x; left node first
  r.fg[2] = face_geo(bl.y, bl.x, br.y, br.x, g.dx);  // S face (y-face j)
  r.fg[3] = face_geo(tl.y, tl.x, tr.y, tr.x, g.dx);  // N face (y-face j+1)
  for (int s = 0; s < 4; ++s) r.vol[s] = fabs(r.fg[s].w * r.fg[s].h);
  // W and S faces: w >= 0 means the donor is the neighbour (this cell receives)
  r.role[0] = r.fg[0].w >= 0.0 ? -1 : 1;
  r.role[1] = r.fg[1].w >= 0.0 ? 1 : -1;
  r.role[2] = r.fg[2].w >= 0.0 ? -1 : 1;
  r.role[3] = r.fg[3].w >= 0.0 ? 1 : -1;
  // corners (§2.3, upwind table of §3.3)
  const NodeD c[4] = {bl, br, tl, tr};
  for (int s = 0; s < 4; ++s) {
    r.vol[4 + s] = fabs(c[s].x * c[s].y);
    const bool sx = c[s].x >= 0.0, sy = c[s].y >= 0.0;
    int role = 0;
    if (s == 0) role = (sx == sy) ? (sx ? -1 : 1) : 0;          // cell is NE of its BL node
    else if (s == 1) role = (sx != sy) ? (sx ? 1 : -1) : 0;     // NW of its BR node
    else if (s == 2) role = (sx != sy) ? (sx ? -1 : 1) : 0;     // SE of its TL node
    else role = (sx == sy) ? (sx ? 1 : -1) : 0;                 // SW of its TR node
    r.role[4 + s] = role;
  }
}

// ------------------------------------------------------------ corrector + geometry (cell)
__global__ void k_remap_cell(Grid g, Fields f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  if (f.s->done) return;
  const double dt = f.s->dt;
  const int C = g.nx * g.ny, q = cidx(g, i, j);
  const int pbl = nidx(g, i, j), pbr = pbl + 1, ptl = pbl + g.nx + 1, ptr = ptl + 1;
  const NodeD bl = node_d(f, pbl, dt), br = node_d(f, pbr, dt), tl = node_d(f, ptl, dt),
              tr = node_d(f, ptr, dt);
  CellRegions r;
  cell_regions(g, bl, br, tl, tr, r);
  // flux-consistent Lagrangian volume: A + outflow - inflow (§2.3)
  double v = g.A;
  for (int s = 0; s < 8; ++s) {
    if (r.role[s] > 0) v += r.vol[s];
    else if (r.role[s] < 0) v -= r.vol[s];
  }
  f.volcf[q] = v;
  if (!(v > 0.0)) atomicOr(&f.s->err, ERR_VOLCF);
  // Vol^{lag} = F(x^n + dt u^{n+1/2})
  const double VL = quad_area(bl.x, bl.y, g.dx + br.x, br.y, tl.x, g.dy + tl.y, g.dx + tr.x,
                              g.dy + tr.y);
  f.VL[q] = VL;
  // Lagrangian centre (mean of the four Lagrangian nodes, relative to the
  // domain origin) and widths
  f.xcL[q] = 0.25 * ((i * g.dx + bl.x) + ((i + 1) * g.dx + br.x) + (i * g.dx + tl.x) +
                     ((i + 1) * g.dx + tr.x));
  f.ycL[q] = 0.25 * ((j * g.dy + bl.y) + (j * g.dy + br.y) + ((j + 1) * g.dy + tl.y) +
                     ((j + 1) * g.dy + tr.y));
  f.dxL[q] = g.dx + 0.5 * ((br.x + tr.x) - (bl.x + tl.x));
  f.dyL[q] = g.dy + 0.5 * ((tl.y + tr.y) - (bl.y + br.y));
  const double Qc = f.Q[q];
  int np = 0, m = -1;
  for (int a = 0; a < g.nmat; ++a) {
    const double V = f.V[a * C + q], M = f.M[a * C + q], E = f.E[a * C + q];
    const double e = M > 0.0 ? E / M : 0.0;
    const double k = V / g.A;
    double eL = e, rcf = 0.0;
    if (present(g, V)) {
      ++np;
      m = a;
      if (!g.kinematic) {
        const double rho = M / V;
        const double rhoL = M / (k * VL);
        eL = e - (f.Ph[a * C + q] + Qc) * (1.0 / rhoL - 1.0 / rho);
      }
      rcf = M / (k * v);
    }
    f.eL[a * C + q] = eL;
    f.rhocf[a * C + q] = rcf;
  }
  f.pure[q] = np == 1 ? m : -1;
}

// ------------------------------------------------------------ reconstruction
// Lagrangian centre and reconstruction data of cell (i,j) seen through the
// walls (mirror cells reflect the centre; scalars are copied).
struct CellView {
  double xc, yc;
  int pure;
};
__device__ __forceinline__ CellView cell_view(const Grid &g, const Fields &f, int i, int j) {
  const int ri = refl_cell(i, g.nx), rj = refl_cell(j, g.ny);
  const int q = cidx(g, ri, rj);
  CellView v;
  v.xc = f.xcL[q];
  v.yc = f.ycL[q];
  if (ri != i) v.xc = (i < 0 ? 0.0 : 2.0 * g.Lx) - v.xc;
  if (rj != j) v.yc = (j < 0 ? 0.0 : 2.0 * g.Ly) - v.yc;
  v.pure = f.pure[q];
  return v;
}
__device__ __forceinline__ double cell_scalar(const Grid &g, const double *a, int i, int j) {
  return a[cidx(g, refl_cell(i, g.nx), refl_cell(j, g.ny))];
}

// Limited slope of a along (si,sj) at cell (i,j), projected on (vx,vy), if the
// donor and both neighbours are pure cells of material m (§4.2); the bool says
// whether order 2 is allowed.
__device__ __forceinline__ bool slope_along(const Grid &g, const Fields &f, const double *a, int i,
                                            int j, int si, int sj, double vx, double vy, int m,
                                            const CellView &cD, double aD, double &slope) {
  const CellView cm = cell_view(g, f, i - si, j - sj), cp = cell_view(g, f, i + si, j + sj);
  if (cm.pure != m || cp.pure != m) return false;
  const double am = cell_scalar(g, a, i - si, j - sj), ap = cell_scalar(g, a, i + si, j + sj);
  const double dm = (aD - am) / ((cD.xc - cm.xc) * vx + (cD.yc - cm.yc) * vy);
  const double dp = (ap - aD) / ((cp.xc - cD.xc) * vx + (cp.yc - cD.yc) * vy);
  slope = van_leer(dm, dp);
  return true;
}

// reconstruction offset (dot the direction) of each region: x, y faces and
// the diagonal corner rules
struct RegionDir {
  int si, sj;
  double vx, vy;
  double off;  // (sgn * width - displacement) . v  (times 1/2 later)
};

// ------------------------------------------------------------ flux kernel
__device__ __forceinline__ void write_region(const Grid &g, double *F, int count, int idx,
                                             double sgn, const double *W, const double *mu,
                                             const double *eps) {
  const int nm = g.nmat;
  double mt = 0.0;
  for (int a = 0; a < nm; ++a) {
    F[a * count + idx] = sgn * W[a];
    F[(nm + a) * count + idx] = sgn * mu[a];
    F[(2 * nm + a) * count + idx] = sgn * eps[a];
    mt += mu[a];
  }
  F[3 * nm * count + idx] = sgn * mt;
}

__device__ __forceinline__ void youngs(const Grid &g, const Fields &f, int a, int i, int j,
                                       double &gx, double &gy) {
  const int C = g.nx * g.ny;
  const double *V = f.V + a * C;
  double k[3][3];
  for (int b = -1; b <= 1; ++b)
    for (int c = -1; c <= 1; ++c) k[b + 1][c + 1] = cell_scalar(g, V, i + c, j + b) / g.A;
  // k[row][col]: row = j offset, col = i offset
  gx = ((k[0][2] + 2.0 * k[1][2] + k[2][2]) - (k[0][0] + 2.0 * k[1][0] + k[2][0])) / (8.0 * g.dx);
  gy = ((k[2][0] + 2.0 * k[2][1] + k[2][2]) - (k[0][0] + 2.0 * k[0][1] + k[0][2])) / (8.0 * g.dy);
}

__global__ void k_flux(Grid g, Fields f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  if (f.s->done) return;
  const double dt = f.s->dt;
  const int nm = g.nmat, C = g.nx * g.ny, q = cidx(g, i, j);
  const int nX = (g.nx + 1) * g.ny, nY = g.nx * (g.ny + 1), nN = (g.nx + 1) * (g.ny + 1);
  const int pbl = nidx(g, i, j), pbr = pbl + 1, ptl = pbl + g.nx + 1, ptr = ptl + 1;
  const NodeD nd[4] = {node_d(f, pbl, dt), node_d(f, pbr, dt), node_d(f, ptl, dt),
                       node_d(f, ptr, dt)};
  CellRegions r;
  cell_regions(g, nd[0], nd[1], nd[2], nd[3], r);
  // region rectangles relative to the Eulerian centre of this cell
  double rx0[8], rx1[8], ry0[8], ry1[8];
  {
    const double hx = 0.5 * g.dx, hy = 0.5 * g.dy;
    // x-faces at x = -hx (W) and +hx (E); rectangle [x_face, x_face + w]
    for (int s = 0; s < 2; ++s) {
      const double xf = s == 0 ? -hx : hx;
      const double w = r.fg[s].w;
      rx0[s] = xf + fmin(0.0, w);
      rx1[s] = xf + fmax(0.0, w);
      ry0[s] = r.fg[s].t0 + (-hy);
      ry1[s] = (r.fg[s].t0 + r.fg[s].h) + (-hy);
    }
    for (int s = 2; s < 4; ++s) {
      const double yf = s == 2 ? -hy : hy;
      const double w = r.fg[s].w;
      ry0[s] = yf + fmin(0.0, w);
      ry1[s] = yf + fmax(0.0, w);
      rx0[s] = r.fg[s].t0 + (-hx);
      rx1[s] = (r.fg[s].t0 + r.fg[s].h) + (-hx);
    }
    const double cx[4] = {-hx, hx, -hx, hx}, cy[4] = {-hy, -hy, hy, hy};
    for (int s = 0; s < 4; ++s) {
      rx0[4 + s] = cx[s] + fmin(0.0, nd[s].x);
      rx1[4 + s] = cx[s] + fmax(0.0, nd[s].x);
      ry0[4 + s] = cy[s] + fmin(0.0, nd[s].y);
      ry1[4 + s] = cy[s] + fmax(0.0, nd[s].y);
    }
  }
  // partial volumes of the outflow regions
  double W[8][MAXMAT];
  int np = 0, pm = -1;
  bool pr[MAXMAT];
  double Vp = 0.0, V[MAXMAT];
  for (int a = 0; a < nm; ++a) {
    V[a] = f.V[a * C + q];
    pr[a] = present(g, V[a]);
    if (pr[a]) {
      ++np;
      pm = a;
      Vp += V[a];
    }
  }
  for (int s = 0; s < 8; ++s)
    for (int a = 0; a < nm; ++a) W[s][a] = 0.0;
  const bool mixed = np >= 2;
  if (!mixed) {
    if (pm >= 0)
      for (int s = 0; s < 8; ++s)
        if (r.role[s] > 0) W[s][pm] = r.vol[s];
  } else {
    // VOF interface on the rectangle through the Lagrangian face midpoints
    // (§4.4), FP64, coordinates centred on the Eulerian cell centre
    const double Rx0 = 0.5 * (nd[0].x + nd[2].x) - 0.5 * g.dx;
    const double Rx1 = 0.5 * (nd[1].x + nd[3].x) + 0.5 * g.dx;
    const double Ry0 = 0.5 * (nd[0].y + nd[1].y) - 0.5 * g.dy;
    const double Ry1 = 0.5 * (nd[2].y + nd[3].y) + 0.5 * g.dy;
    const double gmin = 1e-10 / fmin(g.dx, g.dy);
    double nxv[MAXMAT], nyv[MAXMAT], sv[MAXMAT];
    bool degenerate = false;
    int a0 = -1, b0 = -1;
    if (np == 2) {
      for (int a = 0; a < nm; ++a)
        if (pr[a]) {
          if (a0 < 0) a0 = a;
          else b0 = a;
        }
      double gax, gay, gbx, gby;
      youngs(g, f, a0, i, j, gax, gay);
      youngs(g, f, b0, i, j, gbx, gby);
      const double gx = gax - gbx, gy = gay - gby;
      const double nrm = sqrt(gx * gx + gy * gy);
      if (nrm <= gmin) degenerate = true;
      else {
        nxv[a0] = gx / nrm;
        nyv[a0] = gy / nrm;
        sv[a0] = interface_offset(Rx0, Rx1, Ry0, Ry1, nxv[a0], nyv[a0], V[a0] / Vp);
      }
    } else {
      for (int a = 0; a < nm; ++a) {
        if (!pr[a]) continue;
        double gx, gy;
        youngs(g, f, a, i, j, gx, gy);
        const double nrm = sqrt(gx * gx + gy * gy);
        if (nrm <= gmin) {
          degenerate = true;
          continue;
        }
        nxv[a] = gx / nrm;
        nyv[a] = gy / nrm;
        sv[a] = interface_offset(Rx0, Rx1, Ry0, Ry1, nxv[a], nyv[a], V[a] / Vp);
      }
    }
    for (int s = 0; s < 8; ++s) {
      if (r.role[s] <= 0 || r.vol[s] == 0.0) continue;
      const double vol = r.vol[s];
      if (degenerate) {
        for (int a = 0; a < nm; ++a)
          if (pr[a]) W[s][a] = vol * (V[a] / Vp);
      } else if (np == 2) {
        double wa = rect_halfplane_area(rx0[s], rx1[s], ry0[s], ry1[s], nxv[a0], nyv[a0], sv[a0]);
        wa = fmin(fmax(wa, 0.0), vol);
        W[s][a0] = wa;
        W[s][b0] = vol - wa;
      } else {
        double raw[MAXMAT], sum = 0.0;
        for (int a = 0; a < nm; ++a) {
          raw[a] = pr[a] ? rect_halfplane_area(rx0[s], rx1[s], ry0[s], ry1[s], nxv[a], nyv[a], sv[a])
                         : 0.0;
          sum += raw[a];
        }
        for (int a = 0; a < nm; ++a)
          if (pr[a]) W[s][a] = sum > 0.0 ? vol * (raw[a] / sum) : vol * (V[a] / Vp);
      }
    }
    // donor-side clipping: no material sends more than k_a Vol^{lagCF}; the
    // excess goes to the donor's other present materials by their room
    const double vcf = f.volcf[q];
    double Vcf[MAXMAT], O[MAXMAT], room[MAXMAT], H = 0.0;
    bool over[MAXMAT], any_over = false;
    for (int a = 0; a < nm; ++a) {
      Vcf[a] = (V[a] / g.A) * vcf;
      O[a] = 0.0;
      for (int s = 0; s < 8; ++s)
        if (r.role[s] > 0) O[a] += W[s][a];
      over[a] = pr[a] && O[a] > Vcf[a];
      any_over = any_over || over[a];
    }
    if (any_over) {
      for (int a = 0; a < nm; ++a) {
        room[a] = (pr[a] && !over[a]) ? fmax(0.0, Vcf[a] - O[a]) : 0.0;
        H += room[a];
      }
      if (H > 0.0) {
        for (int s = 0; s < 8; ++s) {
          if (r.role[s] <= 0) continue;
          double freed = 0.0;
          for (int a = 0; a < nm; ++a)
            if (over[a]) {
              const double keep = W[s][a] * (Vcf[a] / O[a]);
              freed += W[s][a] - keep;
              W[s][a] = keep;
            }
          for (int a = 0; a < nm; ++a)
            if (room[a] > 0.0) W[s][a] += freed * (room[a] / H);
        }
      }
    }
  }

  // reconstructed density and energy on each outflow region
  double vr[8][MAXMAT], ve[8][MAXMAT];
  for (int s = 0; s < 8; ++s)
    for (int a = 0; a < nm; ++a) {
      vr[s][a] = f.rhocf[a * C + q];
      ve[s][a] = f.eL[a * C + q];
    }
  if (!mixed && pm >= 0 && g.recon_order == 2) {
    const CellView cD = cell_view(g, f, i, j);
    const double rD = f.rhocf[pm * C + q], eD = f.eL[pm * C + q];
    const double dxL = f.dxL[q], dyL = f.dyL[q];
    const double nrm = sqrt(g.dx * g.dx + g.dy * g.dy);
    double r2[8], e2[8], Mout = 0.0, Eout = 0.0;
    for (int s = 0; s < 8; ++s) {
      r2[s] = rD;
      e2[s] = eD;
      if (r.role[s] <= 0) continue;
      int si, sj;
      double vx, vy, off;
      if (s < 2) {  // x-faces: sgn dx^{lag} - dt u_f
        const double sg = s == 0 ? -1.0 : 1.0;
        const NodeD lo = nd[s == 0 ? 0 : 1], hi = nd[s == 0 ? 2 : 3];
        si = 1; sj = 0; vx = 1.0; vy = 0.0;
        off = sg * dxL - 0.5 * (lo.x + hi.x);
      } else if (s < 4) {
        const double sg = s == 2 ? -1.0 : 1.0;
        const NodeD lo = nd[s == 2 ? 0 : 2], hi = nd[s == 2 ? 1 : 3];
        si = 0; sj = 1; vx = 0.0; vy = 1.0;
        off = sg * dyL - 0.5 * (lo.y + hi.y);
      } else {  // corners: linear diagonal reconstruction (§3.3)
        const NodeD d = nd[s - 4];
        const double sx = d.x >= 0.0 ? 1.0 : -1.0;
        if (corner_main(d)) {
          si = 1; sj = 1; vx = g.dx / nrm; vy = g.dy / nrm;
          off = (sx * dxL - d.x) * vx + (sx * dyL - d.y) * vy;
        } else {
          si = 1; sj = -1; vx = g.dx / nrm; vy = -g.dy / nrm;
          off = (sx * dxL - d.x) * vx + (-sx * dyL - d.y) * vy;
        }
      }
      double sl;
      if (slope_along(g, f, f.rhocf + pm * C, i, j, si, sj, vx, vy, pm, cD, rD, sl)) {
        r2[s] = rD + 0.5 * sl * off;
        slope_along(g, f, f.eL + pm * C, i, j, si, sj, vx, vy, pm, cD, eD, sl);
        e2[s] = eD + 0.5 * sl * off;
      }
      const double mu = r2[s] * W[s][pm];
      Mout += mu;
      Eout += mu * e2[s];
    }
    // positivity guard: the whole donor falls back to upwind values
    const double M = f.M[pm * C + q];
    if (!(Mout > M || Eout > M * eD))
      for (int s = 0; s < 8; ++s) {
        vr[s][pm] = r2[s];
        ve[s][pm] = e2[s];
      }
  }

  // write every region this cell is the donor of, signed along its orientation
  double mu[MAXMAT], eps[MAXMAT];
  for (int s = 0; s < 8; ++s) {
    if (r.role[s] <= 0) continue;
    for (int a = 0; a < nm; ++a) {
      mu[a] = W[s][a] > 0.0 ? vr[s][a] * W[s][a] : 0.0;
      eps[a] = W[s][a] > 0.0 ? mu[a] * ve[s][a] : 0.0;
    }
    switch (s) {
      case 0: write_region(g, f.FX, nX, j * (g.nx + 1) + i, -1.0, W[s], mu, eps); break;
      case 1: write_region(g, f.FX, nX, j * (g.nx + 1) + i + 1, 1.0, W[s], mu, eps); break;
      case 2: write_region(g, f.FY, nY, j * g.nx + i, -1.0, W[s], mu, eps); break;
      case 3: write_region(g, f.FY, nY, (j + 1) * g.nx + i, 1.0, W[s], mu, eps); break;
      case 4: write_region(g, f.FC, nN, pbl, -1.0, W[s], mu, eps); break;  // NE -> SW
      case 5: write_region(g, f.FC, nN, pbr, 1.0, W[s], mu, eps); break;   // NW -> SE
      case 6: write_region(g, f.FC, nN, ptl, -1.0, W[s], mu, eps); break;  // SE -> NW
      default: write_region(g, f.FC, nN, ptr, 1.0, W[s], mu, eps); break;  // SW -> NE
    }
  }
}

// ------------------------------------------------------------ primal update
__global__ void k_update_cell(Grid g, Fields f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  if (f.s->done) return;
  const double dt = f.s->dt;
  const int nm = g.nmat, C = g.nx * g.ny, q = cidx(g, i, j);
  const int nX = (g.nx + 1) * g.ny, nY = g.nx * (g.ny + 1), nN = (g.nx + 1) * (g.ny + 1);
  const int pbl = nidx(g, i, j), pbr = pbl + 1, ptl = pbl + g.nx + 1, ptr = ptl + 1;
  // signed contribution of each region (+: into this cell); walls carry nothing
  int idx[8];
  const double* base[8];
  double sgn[8];
  int cnt[8];
  idx[0] = j * (g.nx + 1) + i;     base[0] = f.FX; sgn[0] = i > 0 ? 1.0 : 0.0;          cnt[0] = nX;
  idx[1] = idx[0] + 1;             base[1] = f.FX; sgn[1] = i < g.nx - 1 ? -1.0 : 0.0; cnt[1] = nX;
  idx[2] = j * g.nx + i;           base[2] = f.FY; sgn[2] = j > 0 ? 1.0 : 0.0;          cnt[2] = nY;
  idx[3] = idx[2] + g.nx;          base[3] = f.FY; sgn[3] = j < g.ny - 1 ? -1.0 : 0.0;  cnt[3] = nY;
  const int pn[4] = {pbl, pbr, ptl, ptr};
  const int In[4] = {i, i + 1, i, i + 1}, Jn[4] = {j, j, j + 1, j + 1};
  const double cs[4] = {1.0, -1.0, 1.0, -1.0};
  for (int s = 0; s < 4; ++s) {
    idx[4 + s] = pn[s];
    base[4 + s] = f.FC;
    cnt[4 + s] = nN;
    const bool wall = In[s] == 0 || In[s] == g.nx || Jn[s] == 0 || Jn[s] == g.ny;
    const bool mainc = corner_main(node_d(f, pn[s], dt));
    // BL, TR corners touch this cell on the main diagonal, BR, TL on the anti
    const bool mine = (s == 0 || s == 3) ? mainc : !mainc;
    sgn[4 + s] = (!wall && mine) ? cs[s] : 0.0;
  }
  double rc2 = 0.0, Msum = 0.0;
  double Vn[MAXMAT], Mn[MAXMAT], En[MAXMAT], Es = 0.0, Ms = 0.0;
  bool bad_nan = false;
  for (int a = 0; a < nm; ++a) {
    const int qa = a * C + q;
    const double M0 = f.M[qa];
    double V = (f.V[qa] / g.A) * f.volcf[q];
    double M = M0;
    double E = M0 * f.eL[qa];
    for (int s = 0; s < 8; ++s) {
      if (sgn[s] == 0.0) continue;
      const double *F = base[s];
      const int c = cnt[s], h = idx[s];
      const double w = F[a * c + h], mu = F[(nm + a) * c + h], ep = F[(2 * nm + a) * c + h];
      if (sgn[s] > 0.0) { V += w; M += mu; E += ep; }
      else { V -= w; M -= mu; E -= ep; }
    }
    f.V[qa] = V;
    f.M[qa] = M;
    f.E[qa] = E;
    Vn[a] = V; Mn[a] = M; En[a] = E;
    Ms += fabs(M);
    Es += fabs(E);
    if (!isfinite(V) || !isfinite(M) || !isfinite(E)) bad_nan = true;
  }
  bool bad_neg = false;
  for (int a = 0; a < nm; ++a) {
    if (Vn[a] < -1e-10 * g.A || Mn[a] < -1e-10 * Ms || En[a] < -1e-10 * Es) bad_neg = true;
    if (present(g, Vn[a])) {
      const double rho = Mn[a] / Vn[a];
      const double e = Mn[a] > 0.0 ? En[a] / Mn[a] : 0.0;
      const double P = (g.gamma[a] - 1.0) * rho * e;
      rc2 += (Vn[a] / g.A) * g.gamma[a] * P;
    }
    Msum += Mn[a];
  }
  if (bad_nan) atomicOr(&f.s->err, ERR_NAN);
  else if (bad_neg) atomicOr(&f.s->err, ERR_NEG);
  const double rhoc = Msum / g.A;
  const double c2 = rhoc > 0.0 ? rc2 / rhoc : 0.0;
  f.cs[q] = c2 > 0.0 ? sqrt(c2) : 0.0;
}

// ------------------------------------------------------------ dual (momentum)
// Nodal data seen through the walls: ghost nodes mirror the velocity (normal
// component negated), the displacement and the Lagrangian position.
struct NodeView {
  double uLx, uLy, dx, dy, X, Y;
};
__device__ __forceinline__ NodeView node_view(const Grid &g, const Fields &f, int I, int J,
                                              double dt) {
  const int rI = refl_node(I, g.nx), rJ = refl_node(J, g.ny);
  const int p = nidx(g, rI, rJ);
  NodeView v;
  v.uLx = f.uLx[p];
  v.uLy = f.uLy[p];
  v.dx = dt * f.uhx[p];
  v.dy = dt * f.uhy[p];
  v.X = rI * g.dx + v.dx;
  v.Y = rJ * g.dy + v.dy;
  if (rI != I) {
    v.uLx = -v.uLx;
    v.dx = -v.dx;
    v.X = (I < 0 ? 0.0 : 2.0 * g.Lx) - v.X;
  }
  if (rJ != J) {
    v.uLy = -v.uLy;
    v.dy = -v.dy;
    v.Y = (J < 0 ? 0.0 : 2.0 * g.Ly) - v.Y;
  }
  return v;
}

// signed total mass flux of x-face (I,j) / y-face (i,J), mirrored at walls
__device__ __forceinline__ double mu_x(const Grid &g, const Fields &f, int I, int j) {
  double sg = 1.0;
  j = refl_cell(j, g.ny);
  if (I < 0) { I = -I; sg = -1.0; }
  else if (I > g.nx) { I = 2 * g.nx - I; sg = -1.0; }
  if (I == 0 || I == g.nx) return 0.0;
  const int nX = (g.nx + 1) * g.ny;
  return sg * f.FX[3 * g.nmat * nX + j * (g.nx + 1) + I];
}
__device__ __forceinline__ double mu_y(const Grid &g, const Fields &f, int i, int J) {
  double sg = 1.0;
  i = refl_cell(i, g.nx);
  if (J < 0) { J = -J; sg = -1.0; }
  else if (J > g.ny) { J = 2 * g.ny - J; sg = -1.0; }
  if (J == 0 || J == g.ny) return 0.0;
  const int nY = g.nx * (g.ny + 1);
  return sg * f.FY[3 * g.nmat * nY + J * g.nx + i];
}
// (main-diagonal, anti-diagonal) signed mass flux of the corner at node (I,J)
__device__ __forceinline__ void mu_corner(const Grid &g, const Fields &f, int I, int J, double dt,
                                          double &dg, double &an) {
  bool fx = false, fy = false;
  if (I < 0) { I = -I; fx = true; }
  else if (I > g.nx) { I = 2 * g.nx - I; fx = true; }
  if (J < 0) { J = -J; fy = true; }
  else if (J > g.ny) { J = 2 * g.ny - J; fy = true; }
  dg = an = 0.0;
  if (I == 0 || I == g.nx || J == 0 || J == g.ny) return;
  const int p = nidx(g, I, J);
  const int nN = (g.nx + 1) * (g.ny + 1);
  const double F = f.FC[3 * g.nmat * nN + p];
  if (corner_main(node_d(f, p, dt))) dg = F;
  else an = F;
  if (fy) { const double t = dg; dg = an; an = t; }
  if (fx) { const double t = dg; dg = -an; an = -t; }
}

__device__ __forceinline__ double dual_wx(const Grid &g, const Fields &f, int I, int J, double dt) {
  return g.dx + 0.5 * (node_view(g, f, I + 1, J, dt).dx - node_view(g, f, I - 1, J, dt).dx);
}
__device__ __forceinline__ double dual_wy(const Grid &g, const Fields &f, int I, int J, double dt) {
  return g.dy + 0.5 * (node_view(g, f, I, J + 1, dt).dy - node_view(g, f, I, J - 1, dt).dy);
}
// limited slopes of both velocity components at node (I,J) along (sI,sJ)
__device__ __forceinline__ void dual_slopes(const Grid &g, const Fields &f, int I, int J, int sI,
                                            int sJ, double vx, double vy, double dt, double &su,
                                            double &sv) {
  const NodeView m = node_view(g, f, I - sI, J - sJ, dt), c = node_view(g, f, I, J, dt),
                 p = node_view(g, f, I + sI, J + sJ, dt);
  const double lm = (c.X - m.X) * vx + (c.Y - m.Y) * vy;
  const double lp = (p.X - c.X) * vx + (p.Y - c.Y) * vy;
  su = van_leer((c.uLx - m.uLx) / lm, (p.uLx - c.uLx) / lp);
  sv = van_leer((c.uLy - m.uLy) / lm, (p.uLy - c.uLy) / lp);
}

struct DualFlux {
  double m, mu, mv;
};
// dual x-face between nodes (I-1,J) and (I,J)
__device__ DualFlux dual_xface(const Grid &g, const Fields &f, int I, int J, double dt) {
  const double phi = 0.25 * (mu_x(g, f, I - 1, J - 1) + mu_x(g, f, I, J - 1) +
                             mu_x(g, f, I - 1, J) + mu_x(g, f, I, J));
  const int D = phi > 0.0 ? I - 1 : I;
  const double sg = phi > 0.0 ? 1.0 : -1.0;
  const NodeView nv = node_view(g, f, D, J, dt);
  double u = nv.uLx, v = nv.uLy;
  if (g.recon_order == 2) {
    const double df = 0.5 * (node_view(g, f, I - 1, J, dt).dx + node_view(g, f, I, J, dt).dx);
    const double off = 0.5 * (sg * dual_wx(g, f, D, J, dt) - df);
    double su, sv;
    dual_slopes(g, f, D, J, 1, 0, 1.0, 0.0, dt, su, sv);
    u += su * off;
    v += sv * off;
  }
  return {phi, phi * u, phi * v};
}
// dual y-face between nodes (I,J-1) and (I,J)
__device__ DualFlux dual_yface(const Grid &g, const Fields &f, int I, int J, double dt) {
  const double phi = 0.25 * (mu_y(g, f, I - 1, J - 1) + mu_y(g, f, I, J - 1) +
                             mu_y(g, f, I - 1, J) + mu_y(g, f, I, J));
  const int D = phi > 0.0 ? J - 1 : J;
  const double sg = phi > 0.0 ? 1.0 : -1.0;
  const NodeView nv = node_view(g, f, I, D, dt);
  double u = nv.uLx, v = nv.uLy;
  if (g.recon_order == 2) {
    const double df = 0.5 * (node_view(g, f, I, J - 1, dt).dy + node_view(g, f, I, J, dt).dy);
    const double off = 0.5 * (sg * dual_wy(g, f, I, D, dt) - df);
    double su, sv;
    dual_slopes(g, f, I, D, 0, 1, 0.0, 1.0, dt, su, sv);
    u += su * off;
    v += sv * off;
  }
  return {phi, phi * u, phi * v};
}
// dual corners at the centre of cell (i,j): main diagonal between nodes
// (i,j) and (i+1,j+1); anti-diagonal between (i,j+1) and (i+1,j)
__device__ DualFlux dual_corner(const Grid &g, const Fields &f, int i, int j, bool anti,
                                double dt) {
  double d00, a00, d10, a10, d01, a01, d11, a11;
  mu_corner(g, f, i, j, dt, d00, a00);
  mu_corner(g, f, i + 1, j, dt, d10, a10);
  mu_corner(g, f, i, j + 1, dt, d01, a01);
  mu_corner(g, f, i + 1, j + 1, dt, d11, a11);
  const double phi = anti ? 0.25 * (a00 + a10 + a01 + a11) : 0.25 * (d00 + d10 + d01 + d11);
  const double sg = phi > 0.0 ? 1.0 : -1.0;
  int DI, DJ;
  if (!anti) { DI = phi > 0.0 ? i : i + 1; DJ = phi > 0.0 ? j : j + 1; }
  else { DI = phi > 0.0 ? i : i + 1; DJ = phi > 0.0 ? j + 1 : j; }
  const NodeView nv = node_view(g, f, DI, DJ, dt);
  double u = nv.uLx, v = nv.uLy;
  if (g.recon_order == 2) {
    const NodeView c00 = node_view(g, f, i, j, dt), c10 = node_view(g, f, i + 1, j, dt),
                   c01 = node_view(g, f, i, j + 1, dt), c11 = node_view(g, f, i + 1, j + 1, dt);
    const double dcx = 0.25 * (c00.dx + c10.dx + c01.dx + c11.dx);
    const double dcy = 0.25 * (c00.dy + c10.dy + c01.dy + c11.dy);
    const double nrm = sqrt(g.dx * g.dx + g.dy * g.dy);
    const double vx = g.dx / nrm, vy = (anti ? -g.dy : g.dy) / nrm;
    const double wx = dual_wx(g, f, DI, DJ, dt), wy = dual_wy(g, f, DI, DJ, dt);
    const double off = anti ? 0.5 * ((sg * wx - dcx) * vx + (-sg * wy - dcy) * vy)
                            : 0.5 * ((sg * wx - dcx) * vx + (sg * wy - dcy) * vy);
    double su, sv;
    dual_slopes(g, f, DI, DJ, 1, anti ? -1 : 1, vx, vy, dt, su, sv);
    u += su * off;
    v += sv * off;
  }
  return {phi, phi * u, phi * v};
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}

__global__ void k_update_node(Grid g, Fields f) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  const bool active = I <= g.nx && J <= g.ny && !f.s->done;
  unsigned long long cand = ~0ull;
  if (active) {
    const double dt = f.s->dt;
    const int p = nidx(g, I, J);
    double ux = f.ux[p], uy = f.uy[p];
    if (!g.kinematic) {
      double m = f.mp[p];
      double mu = m * f.uLx[p], mv = m * f.uLy[p];
      DualFlux d;
      d = dual_xface(g, f, I, J, dt);             m += d.m; mu += d.mu; mv += d.mv;  // W
      d = dual_xface(g, f, I + 1, J, dt);         m -= d.m; mu -= d.mu; mv -= d.mv;  // E
      d = dual_yface(g, f, I, J, dt);             m += d.m; mu += d.mu; mv += d.mv;  // S
      d = dual_yface(g, f, I, J + 1, dt);         m -= d.m; mu -= d.mu; mv -= d.mv;  // N
      d = dual_corner(g, f, I - 1, J - 1, false, dt); m += d.m; mu += d.mu; mv += d.mv;  // SW
      d = dual_corner(g, f, I, J, false, dt);     m -= d.m; mu -= d.mu; mv -= d.mv;  // NE
      d = dual_corner(g, f, I - 1, J, true, dt);  m += d.m; mu += d.mu; mv += d.mv;  // NW
      d = dual_corner(g, f, I, J - 1, true, dt);  m -= d.m; mu -= d.mu; mv -= d.mv;  // SE
      if (!(m > 0.0)) atomicOr(&f.s->err, ERR_NODEMASS);
      ux = mu / m;
      uy = mv / m;
      if (I == 0 || I == g.nx) ux = 0.0;
      if (J == 0 || J == g.ny) uy = 0.0;
      if (!isfinite(ux) || !isfinite(uy)) atomicOr(&f.s->err, ERR_NAN);
      f.ux[p] = ux;
      f.uy[p] = uy;
    }
    // CFL bound of the new state, node-wise: the largest sound speed of the
    // adjacent cells (identical to the cell-wise min over nodes)
    double cmax = 0.0;
    for (int b = -1; b <= 0; ++b)
      for (int a = -1; a <= 0; ++a) {
        const int ci = I + a, cj = J + b;
        if (ci < 0 || cj < 0 || ci >= g.nx || cj >= g.ny) continue;
        cmax = fmax(cmax, f.cs[cidx(g, ci, cj)]);
      }
    const double bound = fmin(g.dx / (cmax + fabs(ux)), g.dy / (cmax + fabs(uy)));
    cand = __double_as_longlong(bound);
  }
  const unsigned long long wmin = wave_min_u64(cand);
  if ((threadIdx.x + threadIdx.y * blockDim.x) % 64 == 0 && wmin != ~0ull)
    atomicMin(&f.s->dtmin, wmin);
}

// CFL bound of the state just set (before the first step)
__global__ void k_sound(Grid g, Fields f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const int C = g.nx * g.ny, q = cidx(g, i, j);
  double rc2 = 0.0, Msum = 0.0;
  for (int a = 0; a < g.nmat; ++a) {
    const double V = f.V[a * C + q], M = f.M[a * C + q], E = f.E[a * C + q];
    if (present(g, V)) {
      const double rho = M / V, e = M > 0.0 ? E / M : 0.0;
      rc2 += (V / g.A) * g.gamma[a] * ((g.gamma[a] - 1.0) * rho * e);
    }
    Msum += M;
  }
  const double rhoc = Msum / g.A;
  const double c2 = rhoc > 0.0 ? rc2 / rhoc : 0.0;
  f.cs[q] = c2 > 0.0 ? sqrt(c2) : 0.0;
}
__global__ void k_dt_nodes(Grid g, Fields f) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  unsigned long long cand = ~0ull;
  if (I <= g.nx && J <= g.ny) {
    const int p = nidx(g, I, J);
    double cmax = 0.0;
    for (int b = -1; b <= 0; ++b)
      for (int a = -1; a <= 0; ++a) {
        const int ci = I + a, cj = J + b;
        if (ci < 0 || cj < 0 || ci >= g.nx || cj >= g.ny) continue;
        cmax = fmax(cmax, f.cs[cidx(g, ci, cj)]);
      }
    const double bound = fmin(g.dx / (cmax + fabs(f.ux[p])), g.dy / (cmax + fabs(f.uy[p])));
    cand = __double_as_longlong(bound);
  }
  const unsigned long long wmin = wave_min_u64(cand);
  if ((threadIdx.x + threadIdx.y * blockDim.x) % 64 == 0 && wmin != ~0ull)
    atomicMin(&f.s->dtmin, wmin);
}

// initial conserved state from (k, rho, e)
__global__ void k_init_state(Grid g, Fields f, const double *k, const double *rho, const double *e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const int C = g.nx * g.ny, q = cidx(g, i, j);
  for (int a = 0; a < g.nmat; ++a) {
    const int h = a * C + q;
    const double V = k[h] * g.A;
    const double M = k[h] > 0.0 ? rho[h] * V : 0.0;
    f.V[h] = V;
    f.M[h] = M;
    f.E[h] = k[h] > 0.0 ? M * e[h] : 0.0;
  }
}

// op 0: start a run (t_end, step_limit) and prepare the first step
// op 1: finish the current step and prepare the next one
__device__ void prepare(const Grid &g, Scalars *s) {
  const double dtmin = __longlong_as_double((long long)s->dtmin);
  double dt = g.fixed_dt > 0.0 ? g.fixed_dt : g.cfl * dtmin;
  s->last = 0;
  if (s->t_end - s->t <= dt) {
    dt = s->t_end - s->t;
    s->last = 1;
  }
  if (!(dt > 0.0) || !isfinite(dt)) {
    s->err |= ERR_DT;
    s->done = 1;
  }
  s->dt = dt;
  s->dtmin = (unsigned long long)__double_as_longlong(INFINITY);
}
__global__ void k_control(Grid g, Scalars *s, int op, double t_end, long long step_limit) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (op == 0) {
    s->t_end = t_end;
    s->step_limit = step_limit;
    s->err = 0;
    s->last = 0;
    s->done = (s->step >= step_limit || !(s->t < t_end)) ? 1 : 0;
    if (!s->done) prepare(g, s);
    return;
  }
  if (s->done) return;
  s->t = s->last ? s->t_end : s->t + s->dt;
  s->step += 1;
  if (s->err || s->last || s->step >= s->step_limit) {
    s->done = 1;
    return;
  }
  prepare(g, s);
}

// derived output fields
__global__ void k_fields(Grid g, Fields f, unsigned bit, double *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int C = g.nx * g.ny;
  if (bit == LR_F_UX || bit == LR_F_UY) {
    if (i > g.nx || j > g.ny) return;
    const int p = nidx(g, i, j);
    out[p] = bit == LR_F_UX ? f.ux[p] : f.uy[p];
    return;
  }
  if (i >= g.nx || j >= g.ny) return;
  const int q = cidx(g, i, j);
  double Ms = 0.0, Es = 0.0, Ps = 0.0;
  for (int a = 0; a < g.nmat; ++a) {
    const double V = f.V[a * C + q], M = f.M[a * C + q], E = f.E[a * C + q];
    const bool pr = present(g, V);
    const double rho = pr ? M / V : 0.0, e = (pr && M > 0.0) ? E / M : 0.0;
    const double P = pr ? (g.gamma[a] - 1.0) * rho * e : 0.0;
    Ms += M;
    Es += E;
    Ps += (V / g.A) * P;
    double v = 0.0;
    bool per = true;
    switch (bit) {
      case LR_F_K: v = V / g.A; break;
      case LR_F_RHOA: v = rho; break;
      case LR_F_EA: v = e; break;
      case LR_F_PA: v = P; break;
      case LR_F_VOL: v = V; break;
      case LR_F_MASS: v = M; break;
      case LR_F_IE: v = E; break;
      default: per = false;
    }
    if (per) out[a * C + q] = v;
  }
  if (bit == LR_F_RHO) out[q] = Ms / g.A;
  if (bit == LR_F_P) out[q] = Ps;
  if (bit == LR_F_E) out[q] = Ms > 0.0 ? Es / Ms : 0.0;
}

// FP64 totals: one partial per block (fixed order), then one block sums them
__global__ void k_totals_partial(Grid g, Fields f, double *part) {
  const int nq = 3 * g.nmat + 3;
  const int C = g.nx * g.ny, N = (g.nx + 1) * (g.ny + 1);
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  const int item = blockIdx.x * blockDim.x + tid;
  for (int qq = 0; qq < nq; ++qq) {
    double v = 0.0;
    if (qq < 3 * g.nmat) {
      const int a = qq % g.nmat, kind = qq / g.nmat;
      const double *src = kind == 0 ? f.V : (kind == 1 ? f.M : f.E);
      if (item < C) v = src[a * C + item];
    } else if (item < N) {
      const int I = item % (g.nx + 1), J = item / (g.nx + 1);
      double m = 0.0;
      for (int b = -1; b <= 0; ++b)
        for (int a = -1; a <= 0; ++a) {
          const int ci = I + a, cj = J + b;
          if (ci < 0 || cj < 0 || ci >= g.nx || cj >= g.ny) continue;
          for (int s = 0; s < g.nmat; ++s) m += 0.25 * f.M[s * C + cidx(g, ci, cj)];
        }
      const double u = f.ux[item], w = f.uy[item];
      const int k = qq - 3 * g.nmat;
      v = k == 0 ? m * u : (k == 1 ? m * w : 0.5 * m * (u * u + w * w));
    }
    sh[tid] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) sh[tid] += sh[tid + o];
      __syncthreads();
    }
    if (tid == 0) part[qq * gridDim.x + blockIdx.x] = sh[0];
    __syncthreads();
  }
}
__global__ void k_totals_final(int nmat, int nb, const double *part, double *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int nq = 3 * nmat + 3;
  for (int qq = 0; qq < nq; ++qq) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[qq * nb + b];
    out[qq] = s;
  }
  // total energy: internal energies plus the nodal kinetic energy
  double et = 0.0;
  for (int a = 0; a < nmat; ++a) et += out[2 * nmat + a];
  out[nq - 1] = et + out[nq - 1];
}

}  // namespace

// =================================================================== host
struct lr_ctx {
  Grid g{};
  Fields f{};
  lr_opts o{};
  hipStream_t own = nullptr, stream = nullptr;
  Scalars *hs = nullptr;  // pinned host mirror of the scalars
  bool have_state = false;
  std::string err;
  std::vector<void *> allocs;
  double *scratch = nullptr;  // staging for outputs, C*nmat doubles at least
  size_t scratch_n = 0;
  // kernel timing (lr_profile): event pairs of the steps of one chunk
  bool prof = false;
  std::vector<hipEvent_t> ev;  // [kChunk][kKernels][2]
  int prof_steps = 0;          // steps recorded in the current chunk
  double prof_ms[16] = {0};
  long prof_n[16] = {0};
};

namespace {

int set_err(lr_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}
#define HIP_CHECK(c, call)                                                          \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      return set_err((c), LR_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

template <class T>
int dalloc(lr_ctx *c, T **p, size_t n) {
  void *q = nullptr;
  if (hipMalloc(&q, (n ? n : 1) * sizeof(T)) != hipSuccess) return LR_ENOMEM;
  c->allocs.push_back(q);
  *p = static_cast<T *>(q);
  return LR_OK;
}

dim3 cell_grid(const Grid &g, dim3 b) {
  return dim3((g.nx + b.x - 1) / b.x, (g.ny + b.y - 1) / b.y);
}
dim3 node_grid(const Grid &g, dim3 b) {
  return dim3((g.nx + 1 + b.x - 1) / b.x, (g.ny + 1 + b.y - 1) / b.y);
}
const dim3 kBlock(64, 4);
constexpr int kChunk = 16;  // steps between completion checks
constexpr int kKernels = 7;
const char *const kKernelNames[kKernels] = {"k_lag_cell",    "k_lag_node",    "k_remap_cell",
                                            "k_flux",        "k_update_cell", "k_update_node",
                                            "k_control"};

int launch_step(lr_ctx *c) {
  const Grid &g = c->g;
  hipStream_t s = c->stream;
  const bool prof = c->prof && c->prof_steps < kChunk;
  hipEvent_t *ev = prof ? &c->ev[(size_t)c->prof_steps * kKernels * 2] : nullptr;
  auto mark = [&](int k, int side) {
    if (prof) (void)hipEventRecord(ev[2 * k + side], s);
  };
  mark(0, 0); k_lag_cell<<<cell_grid(g, kBlock), kBlock, 0, s>>>(g, c->f); mark(0, 1);
  mark(1, 0); k_lag_node<<<node_grid(g, kBlock), kBlock, 0, s>>>(g, c->f); mark(1, 1);
  mark(2, 0); k_remap_cell<<<cell_grid(g, kBlock), kBlock, 0, s>>>(g, c->f); mark(2, 1);
  mark(3, 0); k_flux<<<cell_grid(g, kBlock), kBlock, 0, s>>>(g, c->f); mark(3, 1);
  mark(4, 0); k_update_cell<<<cell_grid(g, kBlock), kBlock, 0, s>>>(g, c->f); mark(4, 1);
  mark(5, 0); k_update_node<<<node_grid(g, kBlock), kBlock, 0, s>>>(g, c->f); mark(5, 1);
  mark(6, 0); k_control<<<1, 1, 0, s>>>(g, c->f.s, 1, 0.0, 0); mark(6, 1);
  if (prof) ++c->prof_steps;
  HIP_CHECK(c, hipGetLastError());
  return LR_OK;
}

// add up the event pairs recorded since the last completion check
int collect_profile(lr_ctx *c) {
  if (!c->prof || c->prof_steps == 0) return LR_OK;
  HIP_CHECK(c, hipStreamSynchronize(c->stream));
  for (int st = 0; st < c->prof_steps; ++st)
    for (int k = 0; k < kKernels; ++k) {
      float ms = 0.0f;
      hipEvent_t *e = &c->ev[((size_t)st * kKernels + k) * 2];
      HIP_CHECK(c, hipEventElapsedTime(&ms, e[0], e[1]));
      c->prof_ms[k] += ms;
      c->prof_n[k] += 1;
    }
  c->prof_steps = 0;
  return LR_OK;
}

int read_scalars(lr_ctx *c) {
  HIP_CHECK(c, hipMemcpyAsync(c->hs, c->f.s, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
  HIP_CHECK(c, hipStreamSynchronize(c->stream));
  return LR_OK;
}

int err_code(lr_ctx *c, int bits) {
  if (bits & ERR_NAN) return set_err(c, LR_ENAN, "non-finite value in the state");
  if (bits & ERR_DT) return set_err(c, LR_EDT, "time step not positive or not finite");
  if (bits & ERR_VOLCF) return set_err(c, LR_ENEGATIVE, "flux-consistent Lagrangian volume <= 0");
  if (bits & ERR_NODEMASS) return set_err(c, LR_ENEGATIVE, "nodal mass <= 0 after remap");
  if (bits & ERR_NEG) return set_err(c, LR_ENEGATIVE, "negative partial volume, mass or energy");
  return LR_OK;
}

// run up to max_steps steps toward t_end, checking completion every `chunk`
int run_steps(lr_ctx *c, double t_end, long long max_steps) {
  read_scalars(c);
  const long long limit = c->hs->step + max_steps;
  k_control<<<1, 1, 0, c->stream>>>(c->g, c->f.s, 0, t_end, limit);
  HIP_CHECK(c, hipGetLastError());
  const int chunk = kChunk;
  for (;;) {
    int rc = read_scalars(c);
    if (rc) return rc;
    rc = collect_profile(c);
    if (rc) return rc;
    if (c->hs->done) break;
    const long long left = c->hs->step_limit - c->hs->step;
    const long long n = left < chunk ? left : chunk;
    for (long long k = 0; k < n; ++k) {
      rc = launch_step(c);
      if (rc) return rc;
    }
  }
  return err_code(c, c->hs->err);
}

}  // namespace

extern "C" {

void lr_default_opts(lr_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->x0 = 0; o->x1 = 1; o->y0 = 0; o->y1 = 1;
  o->cfl = 0.5; o->a1 = 0.5; o->a2 = 1.0;
  o->precision = LR_FP64; o->recon_order = 2; o->kinematic = 0;
  o->k_eps = 1e-10; o->fixed_dt = 0.0;
}

void lr_destroy(lr_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  for (void *p : c->allocs) (void)hipFree(p);
  if (c->hs) (void)hipHostFree(c->hs);
  if (c->own) (void)hipStreamDestroy(c->own);
  delete c;
}

int lr_create(int nx, int ny, int nmat, const lr_eos *eos, const int bc[4], const lr_opts *opts,
              lr_ctx **out) {
  if (!out) return LR_EINVAL;
  *out = nullptr;
  if (nx < 2 || ny < 2 || nmat < 1 || nmat > LR_MAXMAT || !eos) return LR_EINVAL;
  if ((long long)nx * ny > (1ll << 30)) return LR_EINVAL;
  if (bc)
    for (int s = 0; s < 4; ++s)
      if (bc[s] != LR_BC_REFLECT) return LR_EINVAL;
  for (int a = 0; a < nmat; ++a)
    if (!(eos[a].gamma > 1.0) || eos[a].pinf != 0.0) return LR_EINVAL;
  lr_opts o;
  if (opts) o = *opts;
  else lr_default_opts(&o);
  if (!(o.x1 > o.x0) || !(o.y1 > o.y0) || !(o.cfl > 0) || (o.recon_order != 1 && o.recon_order != 2) ||
      !(o.k_eps >= 0) || o.fixed_dt < 0 || o.precision != LR_FP64)
    return LR_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return LR_EDEVICE;
  lr_ctx *c = new (std::nothrow) lr_ctx();
  if (!c) return LR_ENOMEM;
  c->o = o;
  Grid &g = c->g;
  g.nx = nx; g.ny = ny; g.nmat = nmat;
  g.recon_order = o.recon_order; g.kinematic = o.kinematic ? 1 : 0;
  g.dx = (o.x1 - o.x0) / nx; g.dy = (o.y1 - o.y0) / ny; g.A = g.dx * g.dy;
  g.Lx = o.x1 - o.x0; g.Ly = o.y1 - o.y0;
  g.cfl = o.cfl; g.a1 = o.a1; g.a2 = o.a2; g.k_eps = o.k_eps; g.fixed_dt = o.fixed_dt;
  for (int a = 0; a < nmat; ++a) g.gamma[a] = eos[a].gamma;
  const size_t C = (size_t)nx * ny, N = (size_t)(nx + 1) * (ny + 1), m = nmat;
  const size_t nX = (size_t)(nx + 1) * ny, nY = (size_t)nx * (ny + 1), nr = 3 * m + 1;
  Fields &f = c->f;
  int rc = LR_OK;
  rc |= dalloc(c, &f.V, m * C); rc |= dalloc(c, &f.M, m * C); rc |= dalloc(c, &f.E, m * C);
  rc |= dalloc(c, &f.ux, N); rc |= dalloc(c, &f.uy, N);
  rc |= dalloc(c, &f.Q, C); rc |= dalloc(c, &f.S, C); rc |= dalloc(c, &f.Mc, C);
  rc |= dalloc(c, &f.Ph, m * C);
  rc |= dalloc(c, &f.mp, N); rc |= dalloc(c, &f.uhx, N); rc |= dalloc(c, &f.uhy, N);
  rc |= dalloc(c, &f.uLx, N); rc |= dalloc(c, &f.uLy, N);
  rc |= dalloc(c, &f.VL, C); rc |= dalloc(c, &f.volcf, C); rc |= dalloc(c, &f.xcL, C);
  rc |= dalloc(c, &f.ycL, C); rc |= dalloc(c, &f.dxL, C); rc |= dalloc(c, &f.dyL, C);
  rc |= dalloc(c, &f.rhocf, m * C); rc |= dalloc(c, &f.eL, m * C);
  rc |= dalloc(c, &f.pure, C);
  rc |= dalloc(c, &f.FX, nr * nX); rc |= dalloc(c, &f.FY, nr * nY); rc |= dalloc(c, &f.FC, nr * N);
  rc |= dalloc(c, &f.cs, C);
  rc |= dalloc(c, &f.s, 1);
  c->scratch_n = std::max(m * std::max(N, std::max(nX, nY)), (size_t)4096);
  rc |= dalloc(c, &c->scratch, c->scratch_n);
  if (rc != LR_OK || hipHostMalloc((void **)&c->hs, sizeof(Scalars), hipHostMallocDefault) != hipSuccess) {
    lr_destroy(c);
    return LR_ENOMEM;
  }
  if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
    lr_destroy(c);
    return LR_EDEVICE;
  }
  // wall faces and corners are never written by a donor: keep them zero
  if (hipMemsetAsync(f.FX, 0, nr * nX * sizeof(double), c->own) != hipSuccess ||
      hipMemsetAsync(f.FY, 0, nr * nY * sizeof(double), c->own) != hipSuccess ||
      hipMemsetAsync(f.FC, 0, nr * N * sizeof(double), c->own) != hipSuccess ||
      hipStreamSynchronize(c->own) != hipSuccess) {
    lr_destroy(c);
    return LR_EDEVICE;
  }
  c->stream = c->own;
  *out = c;
  return LR_OK;
}

int lr_bind_stream(lr_ctx *c, void *hip_stream) {
  if (!c) return LR_EINVAL;
  HIP_CHECK(c, hipStreamSynchronize(c->stream));
  c->stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->own;
  return LR_OK;
}

int lr_set_state(lr_ctx *c, double t, const double *k, const double *rho, const double *e,
                 const double *ux, const double *uy) {
  if (!c || !k || !rho || !e || !ux || !uy) return LR_EINVAL;
  const Grid &g = c->g;
  const int nx = g.nx, ny = g.ny, nm = g.nmat;
  const size_t C = (size_t)nx * ny, N = (size_t)(nx + 1) * (ny + 1);
  if (!std::isfinite(t)) return set_err(c, LR_EINVAL, "t not finite");
  for (size_t q = 0; q < C; ++q) {
    double ks = 0.0;
    for (int a = 0; a < nm; ++a) {
      const size_t h = a * C + q;
      if (!std::isfinite(k[h]) || !std::isfinite(rho[h]) || !std::isfinite(e[h]))
        return set_err(c, LR_ENAN, "non-finite input");
      if (k[h] < 0.0 || k[h] > 1.0) return set_err(c, LR_ESTATE, "volume fraction outside [0,1]");
      if (k[h] > 0.0 && (!(rho[h] > 0.0) || e[h] < 0.0))
        return set_err(c, LR_ESTATE, "rho <= 0 or e < 0 where k > 0");
      ks += k[h];
    }
    if (std::fabs(ks - 1.0) > 1e-12) return set_err(c, LR_ESTATE, "volume fractions do not sum to 1");
  }
  std::vector<double> u(2 * N);
  for (size_t p = 0; p < N; ++p) {
    if (!std::isfinite(ux[p]) || !std::isfinite(uy[p])) return set_err(c, LR_ENAN, "non-finite velocity");
    const int I = (int)(p % (nx + 1)), J = (int)(p / (nx + 1));
    u[p] = (I == 0 || I == nx) ? 0.0 : ux[p];
    u[N + p] = (J == 0 || J == ny) ? 0.0 : uy[p];
  }
  double *dk = nullptr;
  if (hipMalloc(&dk, 3 * nm * C * sizeof(double)) != hipSuccess) return set_err(c, LR_ENOMEM, "staging");
  hipStream_t s = c->stream;
  int rc = LR_OK;
  do {
    if (hipMemcpyAsync(dk, k, nm * C * sizeof(double), hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(dk + nm * C, rho, nm * C * sizeof(double), hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(dk + 2 * nm * C, e, nm * C * sizeof(double), hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(c->f.ux, u.data(), N * sizeof(double), hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(c->f.uy, u.data() + N, N * sizeof(double), hipMemcpyHostToDevice, s)) {
      rc = set_err(c, LR_EDEVICE, "upload failed");
      break;
    }
    k_init_state<<<cell_grid(g, kBlock), kBlock, 0, s>>>(g, c->f, dk, dk + nm * C, dk + 2 * nm * C);
    Scalars h{};
    h.t = t;
    h.dt = 0.0;
    h.t_end = t;
    const double inf = INFINITY;
    std::memcpy(&h.dtmin, &inf, sizeof inf);
    h.step = 0;
    h.step_limit = 0;
    h.done = 1;
    *c->hs = h;
    if (hipMemcpyAsync(c->f.s, c->hs, sizeof(Scalars), hipMemcpyHostToDevice, s)) {
      rc = set_err(c, LR_EDEVICE, "upload failed");
      break;
    }
    k_sound<<<cell_grid(g, kBlock), kBlock, 0, s>>>(g, c->f);
    k_dt_nodes<<<node_grid(g, kBlock), kBlock, 0, s>>>(g, c->f);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
      rc = set_err(c, LR_EDEVICE, "initialisation kernels failed");
      break;
    }
  } while (0);
  (void)hipFree(dk);
  if (rc == LR_OK) c->have_state = true;
  return rc;
}

int lr_step(lr_ctx *c, double *dt_out) {
  if (!c) return LR_EINVAL;
  if (!c->have_state) return set_err(c, LR_ESTATE, "no state set");
  const int rc = run_steps(c, INFINITY, 1);
  if (dt_out) *dt_out = c->hs->dt;
  return rc;
}

int lr_run(lr_ctx *c, double t_end, long max_steps, long *steps_out, double *t_out) {
  if (!c) return LR_EINVAL;
  if (!c->have_state) return set_err(c, LR_ESTATE, "no state set");
  int rc = read_scalars(c);
  if (rc) return rc;
  if (!(t_end >= c->hs->t) || max_steps < 0) return set_err(c, LR_EINVAL, "t_end < t or max_steps < 0");
  const long long s0 = c->hs->step;
  rc = run_steps(c, t_end, max_steps);
  if (steps_out) *steps_out = (long)(c->hs->step - s0);
  if (t_out) *t_out = c->hs->t;
  return rc;
}

int lr_get_fields(lr_ctx *c, unsigned mask, double *const *out) {
  if (!c || !out) return LR_EINVAL;
  if (!c->have_state) return set_err(c, LR_ESTATE, "no state set");
  const Grid &g = c->g;
  const size_t C = (size_t)g.nx * g.ny, N = (size_t)(g.nx + 1) * (g.ny + 1);
  int slot = 0;
  for (unsigned bit = 1; bit <= LR_F_IE; bit <<= 1) {
    if (!(mask & bit)) continue;
    double *o = out[slot++];
    if (!o) return set_err(c, LR_EINVAL, "null output pointer");
    const bool node = bit == LR_F_UX || bit == LR_F_UY;
    const bool per = bit == LR_F_K || bit == LR_F_RHOA || bit == LR_F_EA || bit == LR_F_PA ||
                     bit == LR_F_VOL || bit == LR_F_MASS || bit == LR_F_IE;
    const size_t n = node ? N : (per ? g.nmat * C : C);
    k_fields<<<node_grid(g, kBlock), kBlock, 0, c->stream>>>(g, c->f, bit, c->scratch);
    HIP_CHECK(c, hipGetLastError());
    HIP_CHECK(c, hipMemcpyAsync(o, c->scratch, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  }
  HIP_CHECK(c, hipStreamSynchronize(c->stream));
  return LR_OK;
}

int lr_totals(lr_ctx *c, double *out) {
  if (!c || !out) return LR_EINVAL;
  if (!c->have_state) return set_err(c, LR_ESTATE, "no state set");
  const Grid &g = c->g;
  const int N = (g.nx + 1) * (g.ny + 1);
  const int nb = (N + 255) / 256, nq = 3 * g.nmat + 3;
  double *part = nullptr;
  HIP_CHECK(c, hipMalloc(&part, ((size_t)nq * nb + nq) * sizeof(double)));
  k_totals_partial<<<nb, 256, 0, c->stream>>>(g, c->f, part);
  k_totals_final<<<1, 64, 0, c->stream>>>(g.nmat, nb, part, part + (size_t)nq * nb);
  hipError_t e1 = hipMemcpyAsync(out, part + (size_t)nq * nb, nq * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream);
  hipError_t e2 = hipStreamSynchronize(c->stream);
  (void)hipFree(part);
  if (e1 != hipSuccess || e2 != hipSuccess) return set_err(c, LR_EDEVICE, "totals failed");
  return LR_OK;
}

int lr_debug_get(lr_ctx *c, const char *name, double *out) {
  if (!c || !name || !out) return LR_EINVAL;
  if (!c->have_state) return set_err(c, LR_ESTATE, "no state set");
  const Grid &g = c->g;
  const Fields &f = c->f;
  const size_t C = (size_t)g.nx * g.ny, N = (size_t)(g.nx + 1) * (g.ny + 1);
  const size_t nX = (size_t)(g.nx + 1) * g.ny, nY = (size_t)g.nx * (g.ny + 1);
  const size_t m = g.nmat;
  std::string n(name);
  auto copy = [&](const void *src, size_t count) -> int {
    HIP_CHECK(c, hipMemcpyAsync(out, src, count * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK(c, hipStreamSynchronize(c->stream));
    return LR_OK;
  };
  if (n == "dt" || n == "t") {
    int rc = read_scalars(c);
    if (rc) return rc;
    out[0] = n == "dt" ? c->hs->dt : c->hs->t;
    return LR_OK;
  }
  if (n == "Q") return copy(f.Q, C);
  if (n == "S") return copy(f.S, C);
  if (n == "volcf") return copy(f.volcf, C);
  if (n == "VL") return copy(f.VL, C);
  if (n == "dxL") return copy(f.dxL, C);
  if (n == "dyL") return copy(f.dyL, C);
  if (n == "eL") return copy(f.eL, m * C);
  if (n == "rhocf") return copy(f.rhocf, m * C);
  if (n == "P_half") return copy(f.Ph, m * C);
  if (n == "mp") return copy(f.mp, N);
  if (n == "uhx") return copy(f.uhx, N);
  if (n == "uhy") return copy(f.uhy, N);
  if (n == "uLx") return copy(f.uLx, N);
  if (n == "uLy") return copy(f.uLy, N);
  if (n == "muX") return copy(f.FX + 3 * m * nX, nX);
  if (n == "muY") return copy(f.FY + 3 * m * nY, nY);
  if (n == "Wpx") return copy(f.FX, m * nX);
  if (n == "Wpy") return copy(f.FY, m * nY);
  if (n == "Wpc") return copy(f.FC, m * N);
  if (n == "dpx" || n == "dpy" || n == "muD" || n == "muA") {
    int rc = read_scalars(c);
    if (rc) return rc;
    const double dt = c->hs->dt;
    std::vector<double> hx(N), hy(N), fc(N);
    HIP_CHECK(c, hipMemcpyAsync(hx.data(), f.uhx, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK(c, hipMemcpyAsync(hy.data(), f.uhy, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK(c, hipMemcpyAsync(fc.data(), f.FC + 3 * m * N, N * sizeof(double), hipMemcpyDeviceToHost,
                                c->stream));
    HIP_CHECK(c, hipStreamSynchronize(c->stream));
    for (size_t p = 0; p < N; ++p) {
      const double dx = dt * hx[p], dy = dt * hy[p];
      const int I = (int)(p % (g.nx + 1)), J = (int)(p / (g.nx + 1));
      const bool wall = I == 0 || I == g.nx || J == 0 || J == g.ny;
      const bool mainc = (dx >= 0.0) == (dy >= 0.0);
      if (n == "dpx") out[p] = dx;
      else if (n == "dpy") out[p] = dy;
      else if (n == "muD") out[p] = (!wall && mainc) ? fc[p] : 0.0;
      else out[p] = (!wall && !mainc) ? fc[p] : 0.0;
    }
    return LR_OK;
  }
  return set_err(c, LR_EINVAL, "unknown stage name");
}

int lr_profile(lr_ctx *c, int enable) {
  if (!c) return LR_EINVAL;
  if (enable && c->ev.empty()) {
    c->ev.resize((size_t)kChunk * kKernels * 2);
    for (auto &e : c->ev) HIP_CHECK(c, hipEventCreate(&e));
  }
  c->prof = enable != 0;
  c->prof_steps = 0;
  return LR_OK;
}

int lr_profile_read(lr_ctx *c, double *ms, long *counts, int n) {
  if (!c || n < 0 || n > kKernels) return LR_EINVAL;
  int rc = collect_profile(c);
  if (rc) return rc;
  for (int k = 0; k < n; ++k) {
    if (ms) ms[k] = c->prof_ms[k];
    if (counts) counts[k] = c->prof_n[k];
  }
  for (int k = 0; k < kKernels; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  return LR_OK;
}

int lr_kernel_count(void) { return kKernels; }

const char *lr_kernel_name(int i) { return (i >= 0 && i < kKernels) ? kKernelNames[i] : ""; }

const char *lr_last_error(const lr_ctx *c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
