// lr_ad.hpp — the alternate-direction (AD) remap, the paper's comparator
// (§2.1.1, §2.1.2, §4.2), on the GPU (part of the lr_kernels.hip translation
// unit).  It replaces the DirectCF remap when the problem's options ask for
// it; the Lagrangian phase is the same.  A step runs two one-dimensional
// passes, X then Y on even steps and Y then X on odd ones (§2.1.2, remark 3);
// each pass remaps the cell and nodal quantities through the faces of its
// direction only:
//   * a face's flux volume is the rectangle of full cell height and width
//     w = mean of the face's two node displacements along the direction;
//   * the pass's Lagrangian volume is A + outflow - inflow of its two faces,
//     its centre and width move along the direction only;
//   * mixed donors place their interface (§4.2: from the pass's own input
//     volume fractions) on the rectangle through the midpoints of the
//     Lagrangian faces of that direction, the others staying Eulerian;
//   * reconstruction, positivity guard, donor-side clipping and the primal
//     update as in DirectCF, on two regions per cell;
//   * the dual (momentum) update through the two dual faces of the direction,
//     each carrying 1/4 of the four same-side primal face mass fluxes.
// The second pass starts from the first pass's state (volume fractions,
// specific energies e = E/M, nodal masses and velocities).
//
// Four kernels per pass over plain global arrays, one thread per cell or
// node: the comparator is not the hot path, so it keeps the simplest data
// flow (no tiles, no staging in LDS).  The mixed-cell arithmetic is FP64 as
// in DirectCF.
#pragma once

namespace {

// direction (0: x, 1: y) of pass `pass` of the step with index `step`
__device__ __forceinline__ int ad_dir(long long step, int pass) {
  const bool xfirst = (step & 1) == 0;
  return ((pass == 0) == xfirst) ? 0 : 1;
}

// displacement d = dt u^{n+1/2} of node (I, J) along `axis`, mirrored
// outside the walls (the normal component changes sign)
template <typename R, typename PT>
__device__ __forceinline__ R ad_disp(const PT &P, R dt, int I, int J, int axis) {
  const int nx = P.g.nx, ny = P.g.ny;
  const int rI = refl_node(I, nx), rJ = refl_node(J, ny);
  const int p = rJ * (nx + 1) + rI;
  R d = dt * ldg((axis == 0 ? P.uhx : P.uhy) + p);
  if ((axis == 0 && rI != I) || (axis == 1 && rJ != J)) d = -d;
  return d;
}

// Lagrangian position of node (I, J) along `axis`: the real node's x + d,
// reflected about the wall for nodes outside it
template <typename R, typename PT>
__device__ __forceinline__ R ad_node_pos(const PT &P, R dt, int I, int J, int axis) {
  const auto &g = P.g;
  const int nx = g.nx, ny = g.ny;
  const int rI = refl_node(I, nx), rJ = refl_node(J, ny);
  const R base = axis == 0 ? R(g.x0) + R(rI) * R(g.dx) : R(g.y0) + R(rJ) * R(g.dy);
  const R v = base + ad_disp(P, dt, rI, rJ, axis);
  if (axis == 0 && rI != I) return R(2) * R(I < 0 ? g.x0 : g.x1) - v;
  if (axis == 1 && rJ != J) return R(2) * R(J < 0 ? g.y0 : g.y1) - v;
  return v;
}

// width w of the pass's face with low node (I, J): x-face (I, j = J) or
// y-face (i = I, J); its volume is |w| times the cell size across
template <typename R, typename PT>
__device__ __forceinline__ R ad_face_w(const PT &P, R dt, int dir, int I, int J) {
  return dir == 0 ? R(0.5) * (ad_disp(P, dt, I, J, 0) + ad_disp(P, dt, I, J + 1, 0))
                  : R(0.5) * (ad_disp(P, dt, I, J, 1) + ad_disp(P, dt, I + 1, J, 1));
}

// index of the pass's face (I, j) [x] or (i, J) [y]
template <typename GT>
__device__ __forceinline__ int ad_face(const GT &g, int dir, int a, int b) {
  return dir == 0 ? b * (g.nx + 1) + a : b * g.nx + a;
}

// the pass's input state: the step's buffer for the first pass, the first
// pass's output for the second
template <typename R>
struct AdIn {
  const R *V, *M, *E;
};
template <typename R, typename PT>
__device__ __forceinline__ AdIn<R> ad_input(const PT &P, int par, int pass) {
  if (pass == 0) return AdIn<R>{P.V[par], P.M[par], P.E[par]};
  return AdIn<R>{P.ad.V, P.ad.M, P.ad.E};
}

// prologue of every AD kernel: the slot of the step, stop flags, dt
template <typename R, typename PT>
__device__ __forceinline__ bool ad_start(const PT &P, int par, R &dt, long long &step) {
  const Slot &S = P.ctl->slot[par];
  const bool stop = (ldg(&S.done) | ldg(&P.ctl->err)) != 0;
  bool last;
  dt = R(slot_dt(P.g, S, last));
  step = ldg(&S.step);
  return stop;
}

// ---- kernel 1 of a pass: per cell, the pass's input fractions, specific
// energies and mixture mass, purity, Lagrangian volume, centre and width
// along the direction, and rho^{lag} = M / (k Vol^{lag}).  The first pass
// also prepares the next step's control slot (as the DirectCF remap does).
template <typename R, int NM>
__global__ void __launch_bounds__(256) k_ad_cells(const Prob<R> *probs, int gpar, int pass) {
  const auto &P = *cst(probs);
  const auto &g = P.g;
  Ctl *ctl = P.ctl;
  const int par = gpar ^ P.flip;
  const Slot &S = ctl->slot[par];
  R dt;
  long long step;
  const bool stop = ad_start(P, par, dt, step);
  const int tid = threadIdx.x;
  if (pass == 0 && blockIdx.x == 0) {
    bool last;
    const double dtd = slot_dt(g, S, last);
    if (stop) {
      if (tid == 0) stg(&ctl->slot[par ^ 1].done, 1);
    } else if (tid < 64) {
      Slot &N = ctl->slot[par ^ 1];
#pragma unroll
      for (int k = 0; k < NDT / 64; ++k)
        if (tid + 64 * k < g.ndt) stg(&N.dtmin[tid + 64 * k], (unsigned long long)__double_as_longlong(INFINITY));
      if (tid == 0) {
        const long long nstep = ldg(&S.step) + 1, limit = ldg(&S.limit);
        const double t = ldg(&S.t), t_end = ldg(&S.t_end);
        stg(&N.t, last ? t_end : t + dtd);
        stg(&N.t_end, t_end);
        stg(&N.step, nstep);
        stg(&N.limit, limit);
        stg(&N.nmix, 0);
        stg(&N.done, (last || nstep >= limit) ? 1 : 0);
        if (!(dtd > 0.0) || !isfinite(dtd)) atomicOr(&ctl->err, ERR_DT);
      }
    }
  }
  if (stop) return;
  const int nx = g.nx, ny = g.ny, C = nx * ny;
  const int q = blockIdx.x * blockDim.x + tid;
  if (q >= C) return;
  const int i = q % nx, j = q / nx;
  const int dir = ad_dir(step, pass);
  const AdIn<R> in = ad_input<R>(P, par, pass);
  const R A = R(g.A);
  R k[NM], Mm[NM], Vm[NM], Msum = R(0);
  int np = 0, pm = -1;
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    const R V = ldg(in.V + (m * C + q)), M = ldg(in.M + (m * C + q));
    Vm[m] = V;
    k[m] = V / A;
    Mm[m] = M;
    const R e = pass == 0 ? ldg(P.eL + (m * C + q)) : (M > R(0) ? ldg(in.E + (m * C + q)) / M : R(0));
    stg(P.ad.k + (m * C + q), k[m]);
    stg(P.ad.e + (m * C + q), e);
    Msum += M;
    if (present(g, V)) {
      ++np;
      pm = m;
    }
  }
  stg(P.ad.Mc + q, Msum);
  stg(P.ad.pure + q, np == 1 ? pm : -1);
  // the two faces of the direction: low (cell is the receiver when w >= 0)
  // and high (cell is the donor when w >= 0), in that order
  const R across = dir == 0 ? R(g.dy) : R(g.dx);
  const R wlo = dir == 0 ? ad_face_w(P, dt, 0, i, j) : ad_face_w(P, dt, 1, i, j);
  const R whi = dir == 0 ? ad_face_w(P, dt, 0, i + 1, j) : ad_face_w(P, dt, 1, i, j + 1);
  R v = A;
  if (wlo >= R(0)) v -= fabs(wlo * across);
  else v += fabs(wlo * across);
  if (whi >= R(0)) v += fabs(whi * across);
  else v -= fabs(whi * across);
  if (!(v > R(0))) atomicOr(&ctl->err, ERR_VOLCF);
  stg(P.ad.vol + q, v);
  // centre and width along the direction (the other coordinate stays Eulerian)
  const R c = R(0.25) * (((ad_node_pos(P, dt, i, j, dir) + ad_node_pos(P, dt, i + 1, j, dir)) +
                          ad_node_pos(P, dt, i, j + 1, dir)) + ad_node_pos(P, dt, i + 1, j + 1, dir));
  const R D = dir == 0 ? R(g.dx) : R(g.dy);
  const R hi_sum = dir == 0 ? ad_disp(P, dt, i + 1, j, 0) + ad_disp(P, dt, i + 1, j + 1, 0)
                            : ad_disp(P, dt, i, j + 1, 1) + ad_disp(P, dt, i + 1, j + 1, 1);
  const R lo_sum = dir == 0 ? ad_disp(P, dt, i, j, 0) + ad_disp(P, dt, i, j + 1, 0)
                            : ad_disp(P, dt, i, j, 1) + ad_disp(P, dt, i + 1, j, 1);
  stg(P.ad.cen + q, c);
  stg(P.ad.wid + q, D + R(0.5) * (hi_sum - lo_sum));
#pragma unroll
  for (int m = 0; m < NM; ++m)
    stg(P.ad.rhocf + (m * C + q), present(g, Vm[m]) ? Mm[m] / (k[m] * v) : R(0));
}

// value of a cell quantity `arr` of donor (i, j) on the pass's face region
// (its face width w, sign sg of the flux along the direction): the donor's
// value, or at order 2 with a pure stencil along the direction the limited
// linear value at the region's centroid (§2.1.1)
template <typename R, typename PT>
__device__ __forceinline__ R ad_recon(const PT &P, const R *arr, int dir, int i, int j, R w, R sg,
                                      int order) {
  const auto &g = P.g;
  const int nx = g.nx, ny = g.ny;
  const int q = j * nx + i;
  const R aD = ldg(arr + q);
  if (order == 1) return aD;
  const int si = dir == 0 ? 1 : 0, sj = 1 - si;
  const int im = refl_cell(i - si, nx), jm = refl_cell(j - sj, ny);
  const int ip = refl_cell(i + si, nx), jp = refl_cell(j + sj, ny);
  const int qm = jm * nx + im, qp = jp * nx + ip;
  const int m = ldg(P.ad.pure + q);
  if (!(m >= 0 && ldg(P.ad.pure + qm) == m && ldg(P.ad.pure + qp) == m)) return aD;
  // centres along the direction; a neighbour outside the walls is the
  // reflection of the cell it mirrors
  const R c = ldg(P.ad.cen + q);
  R cm = ldg(P.ad.cen + qm), cp = ldg(P.ad.cen + qp);
  if (dir == 0) {
    if (i - 1 < 0) cm = R(2) * R(g.x0) - cm;
    if (i + 1 >= nx) cp = R(2) * R(g.x1) - cp;
  } else {
    if (j - 1 < 0) cm = R(2) * R(g.y0) - cm;
    if (j + 1 >= ny) cp = R(2) * R(g.y1) - cp;
  }
  const R d = van_leer_d(aD - ldg(arr + qm), ldg(arr + qp) - aD, c - cm, cp - c);
  return aD + R(0.5) * d * (sg * ldg(P.ad.wid + q) - w);
}

// ---- kernel 2 of a pass: per donor cell, the partial volumes of its
// outflow faces (a pure donor sends its material; a mixed one is split by its
// interface, FP64, then clipped), and their mass and energy fluxes with the
// reconstruction and the positivity guard
template <typename R, int NM>
__global__ void __launch_bounds__(256) k_ad_donor(const Prob<R> *probs, int gpar, int pass) {
  const auto &P = *cst(probs);
  const auto &g = P.g;
  const int par = gpar ^ P.flip;
  R dt;
  long long step;
  if (ad_start(P, par, dt, step)) return;
  const int nx = g.nx, ny = g.ny, C = nx * ny;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= C) return;
  const int i = q % nx, j = q / nx;
  const int dir = ad_dir(step, pass);
  const AdIn<R> in = ad_input<R>(P, par, pass);
  const int nF = dir == 0 ? (nx + 1) * ny : nx * (ny + 1);
  const R across = dir == 0 ? R(g.dy) : R(g.dx);
  // the two faces: 0 low, 1 high; the cell is the donor of the low face when
  // w < 0 and of the high face when w >= 0
  R w[2];
  int fidx[2];
  bool out[2];
  w[0] = ad_face_w(P, dt, dir, i, j);
  w[1] = dir == 0 ? ad_face_w(P, dt, 0, i + 1, j) : ad_face_w(P, dt, 1, i, j + 1);
  fidx[0] = ad_face(g, dir, i, j);
  fidx[1] = dir == 0 ? ad_face(g, 0, i + 1, j) : ad_face(g, 1, i, j + 1);
  out[0] = !(w[0] >= R(0));
  out[1] = w[1] >= R(0);
  if (!out[0] && !out[1]) return;
  R vol[2];
  for (int f = 0; f < 2; ++f) vol[f] = fabs(w[f] * across);
  const int pure = ldg(P.ad.pure + q);
  R W[2][NM];
#pragma unroll
  for (int f = 0; f < 2; ++f)
#pragma unroll
    for (int m = 0; m < NM; ++m) W[f][m] = R(0);
  if (pure >= 0) {
    for (int f = 0; f < 2; ++f)
      if (out[f])
#pragma unroll
        for (int m = 0; m < NM; ++m)
          if (m == pure) W[f][m] = vol[f];
  } else {
    // §4.4 on the pass's Lagrangian cell, FP64
    const double hx = 0.5 * g.dx, hy = 0.5 * g.dy;
    const double dbl = dir == 0 ? double(ad_disp(P, dt, i, j, 0)) : double(ad_disp(P, dt, i, j, 1));
    const double dbr = dir == 0 ? double(ad_disp(P, dt, i + 1, j, 0)) : double(ad_disp(P, dt, i + 1, j, 1));
    const double dtl = dir == 0 ? double(ad_disp(P, dt, i, j + 1, 0)) : double(ad_disp(P, dt, i, j + 1, 1));
    const double dtr = dir == 0 ? double(ad_disp(P, dt, i + 1, j + 1, 0))
                                : double(ad_disp(P, dt, i + 1, j + 1, 1));
    const double Rx0 = (dir == 0 ? 0.5 * (dbl + dtl) : 0.0) - hx;
    const double Rx1 = (dir == 0 ? 0.5 * (dbr + dtr) : 0.0) + hx;
    const double Ry0 = (dir == 1 ? 0.5 * (dbl + dbr) : 0.0) - hy;
    const double Ry1 = (dir == 1 ? 0.5 * (dtl + dtr) : 0.0) + hy;
    double V[NM], Vp = 0.0;
    bool pr[NM];
    int np = 0, a0 = -1, b0 = -1;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      V[m] = double(ldg(in.V + (m * C + q)));
      pr[m] = V[m] > g.k_eps * g.A;
      if (pr[m]) {
        ++np;
        Vp += V[m];
        if (a0 < 0) a0 = m;
        else if (b0 < 0) b0 = m;
      }
    }
    const double gmin = 1e-10 / fmin(g.dx, g.dy);
    // Youngs gradients of the pass's input fractions (3 x 3, mirrored)
    double GX[NM], GY[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      double kk[3][3];
      for (int bb = 0; bb < 3; ++bb)
        for (int aa = 0; aa < 3; ++aa)
          kk[bb][aa] = double(ldg(P.ad.k + (m * C + refl_cell(j + bb - 1, ny) * nx + refl_cell(i + aa - 1, nx))));
      GX[m] = ((kk[0][2] + 2.0 * kk[1][2] + kk[2][2]) - (kk[0][0] + 2.0 * kk[1][0] + kk[2][0])) / (8.0 * g.dx);
      GY[m] = ((kk[2][0] + 2.0 * kk[2][1] + kk[2][2]) - (kk[0][0] + 2.0 * kk[0][1] + kk[0][2])) / (8.0 * g.dy);
    }
    double NX[NM], NY[NM], OF[NM];
    bool degenerate = false;
#pragma unroll
    for (int m = 0; m < NM; ++m) NX[m] = NY[m] = OF[m] = 0.0;
    if (np == 2) {
      double gx = 0.0, gy = 0.0, Va = 0.0;
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        if (m == a0) { gx += GX[m]; gy += GY[m]; Va = V[m]; }
      }
#pragma unroll
      for (int m = 0; m < NM; ++m)
        if (m == b0) { gx = gx - GX[m]; gy = gy - GY[m]; }
      const double nrm = sqrt(gx * gx + gy * gy);
      if (nrm <= gmin) degenerate = true;
      else {
#pragma unroll
        for (int m = 0; m < NM; ++m)
          if (m == a0) {
            NX[m] = gx / nrm;
            NY[m] = gy / nrm;
            OF[m] = interface_offset(Rx0, Rx1, Ry0, Ry1, NX[m], NY[m], Va / Vp);
          }
      }
    } else {
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        if (!pr[m]) continue;
        const double nrm = sqrt(GX[m] * GX[m] + GY[m] * GY[m]);
        if (nrm <= gmin) {
          degenerate = true;
          continue;
        }
        NX[m] = GX[m] / nrm;
        NY[m] = GY[m] / nrm;
        OF[m] = interface_offset(Rx0, Rx1, Ry0, Ry1, NX[m], NY[m], V[m] / Vp);
      }
    }
    double Wd[2][NM];
    for (int f = 0; f < 2; ++f) {
#pragma unroll
      for (int m = 0; m < NM; ++m) Wd[f][m] = 0.0;
      const double vf = double(vol[f]);
      if (!out[f] || vf == 0.0) continue;
      // the face's flux rectangle in the frame of the donor's centre
      const double wf = double(w[f]);
      double x0, x1, y0, y1;
      const double side = f == 0 ? -0.5 : 0.5;
      if (dir == 0) {
        x0 = fmin(0.0, wf) + side * g.dx;
        x1 = fmax(0.0, wf) + side * g.dx;
        y0 = 0.0 + (-0.5 * g.dy);
        y1 = g.dy + (-0.5 * g.dy);
      } else {
        x0 = 0.0 + (-0.5 * g.dx);
        x1 = g.dx + (-0.5 * g.dx);
        y0 = fmin(0.0, wf) + side * g.dy;
        y1 = fmax(0.0, wf) + side * g.dy;
      }
      if (degenerate) {
#pragma unroll
        for (int m = 0; m < NM; ++m)
          if (pr[m]) Wd[f][m] = vf * (V[m] / Vp);
      } else if (np == 2) {
        double wa = 0.0;
#pragma unroll
        for (int m = 0; m < NM; ++m)
          if (m == a0) wa = rect_halfplane_area(x0, x1, y0, y1, NX[m], NY[m], OF[m]);
        wa = fmin(fmax(wa, 0.0), vf);
#pragma unroll
        for (int m = 0; m < NM; ++m) {
          if (m == a0) Wd[f][m] = wa;
          if (m == b0) Wd[f][m] = vf - wa;
        }
      } else {
        double raw[NM], sum = 0.0;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
          raw[m] = pr[m] ? rect_halfplane_area(x0, x1, y0, y1, NX[m], NY[m], OF[m]) : 0.0;
          sum += raw[m];
        }
#pragma unroll
        for (int m = 0; m < NM; ++m)
          if (pr[m]) Wd[f][m] = sum > 0.0 ? vf * (raw[m] / sum) : vf * (V[m] / Vp);
      }
    }
    // donor-side clipping against k_m Vol^{lag} of the pass
    const double vlag = double(ldg(P.ad.vol + q));
    double Vcf[NM], O[NM], room[NM], H = 0.0;
    bool over[NM], any_over = false;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      Vcf[m] = double(ldg(P.ad.k + (m * C + q))) * vlag;
      O[m] = 0.0;
      for (int f = 0; f < 2; ++f)
        if (out[f]) O[m] += Wd[f][m];
      over[m] = pr[m] && O[m] > Vcf[m];
      any_over = any_over || over[m];
    }
    if (any_over) {
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        room[m] = (pr[m] && !over[m]) ? fmax(0.0, Vcf[m] - O[m]) : 0.0;
        H += room[m];
      }
      if (H > 0.0)
        for (int f = 0; f < 2; ++f) {
          if (!out[f]) continue;
          double freed = 0.0;
#pragma unroll
          for (int m = 0; m < NM; ++m)
            if (over[m]) {
              const double keep = Wd[f][m] * (Vcf[m] / O[m]);
              freed += Wd[f][m] - keep;
              Wd[f][m] = keep;
            }
#pragma unroll
          for (int m = 0; m < NM; ++m)
            if (room[m] > 0.0) Wd[f][m] += freed * (room[m] / H);
        }
    }
    for (int f = 0; f < 2; ++f)
#pragma unroll
      for (int m = 0; m < NM; ++m) W[f][m] = R(Wd[f][m]);
  }
  // reconstruction and fluxes; a mixed donor stays at order 1 (§4.2); the
  // positivity guard sends a pure donor back to order 1
  int order = g.recon_order;
  if (pure < 0) order = 1;
  R mu[2][NM], ep[2][NM];
  for (int pass2 = 0; pass2 < 2; ++pass2) {
    R Mout[NM], Eout[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) Mout[m] = Eout[m] = R(0);
    for (int f = 0; f < 2; ++f) {
      const R sg = w[f] >= R(0) ? R(1) : R(-1);
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        mu[f][m] = ep[f][m] = R(0);
        if (!out[f] || !(W[f][m] > R(0))) continue;
        const R rho = ad_recon(P, P.ad.rhocf + m * C, dir, i, j, w[f], sg, order);
        const R e = ad_recon(P, P.ad.e + m * C, dir, i, j, w[f], sg, order);
        mu[f][m] = rho * W[f][m];
        ep[f][m] = mu[f][m] * e;
        Mout[m] += mu[f][m];
        Eout[m] += ep[f][m];
      }
    }
    if (order == 1) break;
    R Mp = R(0), Ep = R(0), Mo = R(0), Eo = R(0);
#pragma unroll
    for (int m = 0; m < NM; ++m)
      if (m == pure) {
        Mp = ldg(in.M + (m * C + q));
        Ep = Mp * ldg(P.ad.e + (m * C + q));
        Mo = Mout[m];
        Eo = Eout[m];
      }
    if (!(Mo > Mp || Eo > Ep)) break;
    order = 1;
  }
  for (int f = 0; f < 2; ++f) {
    if (!out[f]) continue;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      stg(P.ad.W + (m * nF + fidx[f]), W[f][m]);
      stg(P.ad.mu + (m * nF + fidx[f]), mu[f][m]);
      stg(P.ad.eps + (m * nF + fidx[f]), ep[f][m]);
    }
  }
}

// ---- kernel 3 of a pass: the primal update of each cell from its low then
// high face (V = k Vol^{lag} + in - out, M = M + in - out, E = M e + in - out),
// the signed total mass flux of its low face (and of the wall face at the
// far end), and the checks; the second pass also forms the sound speed of
// the new state for the CFL bound
template <typename R, int NM>
__global__ void __launch_bounds__(256) k_ad_update(const Prob<R> *probs, int gpar, int pass) {
  const auto &P = *cst(probs);
  const auto &g = P.g;
  Ctl *ctl = P.ctl;
  const int par = gpar ^ P.flip;
  R dt;
  long long step;
  if (ad_start(P, par, dt, step)) return;
  const int nx = g.nx, ny = g.ny, C = nx * ny;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= C) return;
  const int i = q % nx, j = q / nx;
  const int dir = ad_dir(step, pass);
  const AdIn<R> in = ad_input<R>(P, par, pass);
  const int nF = dir == 0 ? (nx + 1) * ny : nx * (ny + 1);
  R *Vd = pass == 0 ? P.ad.V : P.V[par ^ 1];
  R *Md = pass == 0 ? P.ad.M : P.M[par ^ 1];
  R *Ed = pass == 0 ? P.ad.E : P.E[par ^ 1];
  const int flo = ad_face(g, dir, i, j);
  const int fhi = dir == 0 ? ad_face(g, 0, i + 1, j) : ad_face(g, 1, i, j + 1);
  const bool wall_lo = dir == 0 ? i == 0 : j == 0;
  const bool wall_hi = dir == 0 ? i == nx - 1 : j == ny - 1;
  // roles: the low face brings material in when w >= 0, the high face when w < 0
  const R wlo = ad_face_w(P, dt, dir, i, j);
  const R whi = dir == 0 ? ad_face_w(P, dt, 0, i + 1, j) : ad_face_w(P, dt, 1, i, j + 1);
  const R slo = wall_lo ? R(0) : (wlo >= R(0) ? R(1) : R(-1));
  const R shi = wall_hi ? R(0) : (whi >= R(0) ? R(-1) : R(1));
  const R vol = ldg(P.ad.vol + q);
  const R A = R(g.A);
  R Vn[NM], Mn[NM], En[NM], Msa = R(0), Esa = R(0), mlo = R(0);
  bool bad_nan = false;
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    const R M0 = ldg(in.M + (m * C + q));
    R V = ldg(P.ad.k + (m * C + q)) * vol, M = M0, E = M0 * ldg(P.ad.e + (m * C + q));
    if (slo != R(0)) {
      const R Wf = ldg(P.ad.W + (m * nF + flo)), mf = ldg(P.ad.mu + (m * nF + flo)),
              ef = ldg(P.ad.eps + (m * nF + flo));
      if (slo > R(0)) { V += Wf; M += mf; E += ef; }
      else { V -= Wf; M -= mf; E -= ef; }
      mlo += mf;
    }
    if (shi != R(0)) {
      const R Wf = ldg(P.ad.W + (m * nF + fhi)), mf = ldg(P.ad.mu + (m * nF + fhi)),
              ef = ldg(P.ad.eps + (m * nF + fhi));
      if (shi > R(0)) { V += Wf; M += mf; E += ef; }
      else { V -= Wf; M -= mf; E -= ef; }
    }
    Vn[m] = V;
    Mn[m] = M;
    En[m] = E;
    stg(Vd + (m * C + q), V);
    stg(Md + (m * C + q), M);
    stg(Ed + (m * C + q), E);
    Msa += fabs(M);
    Esa += fabs(E);
    if (!isfinite(V) || !isfinite(M) || !isfinite(E)) bad_nan = true;
  }
  // signed total mass flux of the low face (zero on the wall) and of the
  // wall face at the far end
  stg(P.ad.muF + flo, wall_lo ? R(0) : (wlo >= R(0) ? mlo : -mlo));
  if (wall_hi) stg(P.ad.muF + fhi, R(0));
  bool bad_neg = false;
  R rc2 = R(0), Msum = R(0);
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    const R tol = R(-g.neg_tol);
    if (Vn[m] < tol * A || Mn[m] < tol * Msa || En[m] < tol * Esa) bad_neg = true;
    if (pass == 1 && present(g, Vn[m])) {
      const R rho = qdiv(Mn[m], Vn[m]);
      const R e = Mn[m] > R(0) ? qdiv(En[m], Mn[m]) : R(0);
      rc2 += eos_krc2(g, m, qdiv(Vn[m], A), eos_p(g, m, rho, e));
    }
    Msum += Mn[m];
  }
  if (bad_nan) atomicOr(&ctl->err, ERR_NAN);
  else if (bad_neg) atomicOr(&ctl->err, ERR_NEG);
  if (pass == 1) {
    const R rhoc = qdiv(Msum, A);
    const R c2 = rhoc > R(0) ? qdiv(rc2, rhoc) : R(0);
    stg(P.cs + q, c2 > R(0) ? sqrt(c2) : R(0));
  }
}

// signed mass flux of the pass's face (a, b) (x-face (I, j) or y-face
// (i, J)) for any index around the grid: faces beyond a wall mirror the real
// face with the normal flux negated
template <typename R, typename PT>
__device__ __forceinline__ R ad_face_flux(const PT &P, int dir, int a, int b) {
  const auto &g = P.g;
  if (dir == 0) {
    const int rI = refl_node(a, g.nx), rj = refl_cell(b, g.ny);
    const R v = ldg(P.ad.muF + (rj * (g.nx + 1) + rI));
    return rI != a ? -v : v;
  }
  const int ri = refl_cell(a, g.nx), rJ = refl_node(b, g.ny);
  const R v = ldg(P.ad.muF + (rJ * g.nx + ri));
  return rJ != b ? -v : v;
}

// velocity component `axis` of the pass's input at node (I, J), mirrored
template <typename R, typename PT>
__device__ __forceinline__ R ad_vel(const PT &P, int pass, int I, int J, int axis) {
  const int nx = P.g.nx, ny = P.g.ny;
  const int rI = refl_node(I, nx), rJ = refl_node(J, ny);
  const int p = rJ * (nx + 1) + rI;
  const R *u = pass == 0 ? (axis == 0 ? P.uLx : P.uLy) : (axis == 0 ? P.ad.ux : P.ad.uy);
  R v = ldg(u + p);
  if ((axis == 0 && rI != I) || (axis == 1 && rJ != J)) v = -v;
  return v;
}

// mass, x- and y-momentum through the pass's dual face between nodes
// (I - sI, J - sJ) and (I, J): 1/4 of the four same-side primal face mass
// fluxes, upwind donor node, velocity reconstructed along the direction
// (dual centres at the Lagrangian node positions)
template <typename R, typename PT>
__device__ __forceinline__ void ad_dual_face(const PT &P, R dt, int pass, int dir, int I, int J, R &fm,
                                             R &fu, R &fv) {
  const auto &g = P.g;
  R phi;
  if (dir == 0)
    phi = R(0.25) * (((ad_face_flux<R>(P, 0, I - 1, J - 1) + ad_face_flux<R>(P, 0, I, J - 1)) +
                      ad_face_flux<R>(P, 0, I - 1, J)) + ad_face_flux<R>(P, 0, I, J));
  else
    phi = R(0.25) * (((ad_face_flux<R>(P, 1, I - 1, J - 1) + ad_face_flux<R>(P, 1, I, J - 1)) +
                      ad_face_flux<R>(P, 1, I - 1, J)) + ad_face_flux<R>(P, 1, I, J));
  const int sI = dir == 0 ? 1 : 0, sJ = 1 - sI;
  const bool fwd = phi > R(0);
  const int DI = fwd ? I - sI : I, DJ = fwd ? J - sJ : J;
  const R sg = fwd ? R(1) : R(-1);
  R vu = ad_vel<R>(P, pass, DI, DJ, 0), vv = ad_vel<R>(P, pass, DI, DJ, 1);
  if (g.recon_order == 2) {
    const R D = dir == 0 ? R(g.dx) : R(g.dy);
    const R df = R(0.5) * (ad_disp(P, dt, I - sI, J - sJ, dir) + ad_disp(P, dt, I, J, dir));
    const R wdual = D + R(0.5) * (ad_disp(P, dt, DI + sI, DJ + sJ, dir) - ad_disp(P, dt, DI - sI, DJ - sJ, dir));
    const R off = R(0.5) * (sg * wdual - df);
    const R xc = ad_node_pos(P, dt, DI, DJ, dir);
    const R lm = xc - ad_node_pos(P, dt, DI - sI, DJ - sJ, dir);
    const R lp = ad_node_pos(P, dt, DI + sI, DJ + sJ, dir) - xc;
    const R um = ad_vel<R>(P, pass, DI - sI, DJ - sJ, 0), up = ad_vel<R>(P, pass, DI + sI, DJ + sJ, 0);
    const R wm = ad_vel<R>(P, pass, DI - sI, DJ - sJ, 1), wp = ad_vel<R>(P, pass, DI + sI, DJ + sJ, 1);
    const R uD = vu, wD = vv;
    vu = uD + van_leer_d(uD - um, up - uD, lm, lp) * off;
    vv = wD + van_leer_d(wD - wm, wp - wD, lm, lp) * off;
  }
  fm = phi;
  fu = phi * vu;
  fv = phi * vv;
}

// ---- kernel 4 of a pass: per node, the momentum update through the low and
// high dual faces of the direction (m u = m_p u + in - out, m_p = 1/4 of the
// pass input's adjacent cell masses), the wall-normal component zeroed; the
// second pass then folds the node-wise CFL bound of the new state into the
// next step's slot.  Kinematic problems keep their prescribed velocity.
template <typename R, int NM>
__global__ void __launch_bounds__(256) k_ad_dual(const Prob<R> *probs, int gpar, int pass) {
  const auto &P = *cst(probs);
  const auto &g = P.g;
  Ctl *ctl = P.ctl;
  const int par = gpar ^ P.flip;
  R dt;
  long long step;
  if (ad_start(P, par, dt, step)) return;
  const int nx = g.nx, ny = g.ny;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long cand = ~0ull;
  if (p < (nx + 1) * (ny + 1)) {
    const int I = p % (nx + 1), J = p / (nx + 1);
    R ux, uy;
    if (!g.kinematic) {
      const int dir = ad_dir(step, pass);
      const int sI = dir == 0 ? 1 : 0, sJ = 1 - sI;
      R mp;
      {
        auto Mc = [&](int a, int b) { return ldg(P.ad.Mc + (refl_cell(b, ny) * nx + refl_cell(a, nx))); };
        mp = R(0.25) * (((Mc(I - 1, J - 1) + Mc(I, J - 1)) + Mc(I - 1, J)) + Mc(I, J));
      }
      R flm, flu, flv, fhm, fhu, fhv;
      ad_dual_face(P, dt, pass, dir, I, J, flm, flu, flv);
      ad_dual_face(P, dt, pass, dir, I + sI, J + sJ, fhm, fhu, fhv);
      R m = mp, mu = mp * ad_vel<R>(P, pass, I, J, 0), mv = mp * ad_vel<R>(P, pass, I, J, 1);
      m += flm; mu += flu; mv += flv;
      m -= fhm; mu -= fhu; mv -= fhv;
      if (!(m > R(0))) atomicOr(&ctl->err, ERR_NODEMASS);
      ux = mu / m;
      uy = mv / m;
      if (I == 0 || I == nx) ux = R(0);
      if (J == 0 || J == ny) uy = R(0);
      if (!isfinite(ux) || !isfinite(uy)) atomicOr(&ctl->err, ERR_NAN);
      stg((pass == 0 ? P.ad.ux : P.ux) + p, ux);
      stg((pass == 0 ? P.ad.uy : P.uy) + p, uy);
    } else {
      ux = ldg(P.ux + p);
      uy = ldg(P.uy + p);
    }
    if (pass == 1) {
      R cmax = R(0);
      for (int bb = -1; bb <= 0; ++bb)
        for (int aa = -1; aa <= 0; ++aa) {
          const int ci = I + aa, cj = J + bb;
          if (ci < 0 || cj < 0 || ci >= nx || cj >= ny) continue;
          cmax = fmax(cmax, ldg(P.cs + (cj * nx + ci)));
        }
      const double bound = fmin(double(R(g.dx) / (cmax + fabs(ux))), double(R(g.dy) / (cmax + fabs(uy))));
      cand = (unsigned long long)__double_as_longlong(bound);
    }
  }
  if (pass == 1) block_min_to_slot(cand, ctl->slot[par ^ 1], g.ndt);
}

// one step with the AD remap: the Lagrangian phase, then the two passes
template <typename R, int NM>
void ad_step_impl(const Launch &L, int gpar, hipStream_t s, hipEvent_t *ev) {
  const Prob<R> *p = static_cast<const Prob<R> *>(L.probs);
  const unsigned cb = (unsigned)((L.cells + 255) / 256), nb = (unsigned)((L.nodes + 255) / 256);
  bool wide = false;
  if constexpr (sizeof(R) == 8) {
    wide = L.cell_blocks <= kWideMaxTiles;
    if (wide)
      launch_b(k_lagrange<R, NM, false, true, TileDefault>, dim3(L.cell_blocks), 2 * NTHREADS, s, ev, p,
               L.cell_map, L.cell_blocks, gpar);
  }
  if (!wide)
    launch(k_lagrange<R, NM, false, false, TileDefault>, dim3(L.cell_blocks), s, ev, p, L.cell_map, L.cell_blocks,
           gpar);
  for (int pass = 0; pass < 2; ++pass) {
    k_ad_cells<R, NM><<<cb, 256, 0, s>>>(p, gpar, pass);
    k_ad_donor<R, NM><<<cb, 256, 0, s>>>(p, gpar, pass);
    k_ad_update<R, NM><<<cb, 256, 0, s>>>(p, gpar, pass);
    k_ad_dual<R, NM><<<nb, 256, 0, s>>>(p, gpar, pass);
  }
}

}  // namespace
