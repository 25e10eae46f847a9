// lr_step.hpp — HIP kernels (gfx950) of one DirectCF Lagrange–Remap time
// step (B. Chaudet, arXiv:2208.13409), templated on the bulk precision R
// (double, or float with FP64 islands), the number of materials NM and the
// tile shape T.  Included by one translation unit per tile shape.
//
// A step is four launches, each over a whole batch of problems (a block map
// gives every block its problem and tile, 32x8 cells by default; the
// mixed-cell kernel has a grid of list chunks x problems; small FP64 launches
// on 32x8 and 32x12 tiles run the Lagrange and dual tiles with two threads per
// cell or node, the others with one thread per cell of the tile):
//   k_lagrange  cell tiles: predictor per cell staged in LDS (EOS, Wilkins Q,
//               Vol^{n+1/2}, P_a^{n+1/2}; §1.2, §4.1), nodal mass and gradient
//               of P+Q, u^{n+1/2}, u^{lag} of the tile's nodes; corrector
//               energies e_a^{lag} of its cells; the tile's mixed cells join a
//               compact list
//   k_mixed     the problems' compact lists of mixed cells (FP64, eight
//               lanes per cell, spread over the device): Youngs normal,
//               interface on the rectangular approximation of the Lagrangian
//               cell, partial volumes of the outflow regions, donor-side
//               clipping (§4.4)
//   k_remap     cell tiles: node displacements, face volumes and cell records
//               (Vol^{lagCF}, rho^{lagCF}, centres) staged in LDS with
//               a two-cell halo; each flux region's order-2 values formed once
//               (reconstruction §2.1.1, §3.3, §4.2), the positivity guard per
//               donor; each cell then gathers its nine-point update (§2.3,
//               §4.4); compensated sums in FP32
//   k_dual      node tiles: dual face and corner mass fluxes (1/4-averages),
//               reconstructed velocities, each dual region once in LDS; nodal
//               momentum update; wavefront-shuffle min of the next CFL bound
// The conserved state is double-buffered (the remap reads step n's buffer
// while neighbouring tiles write step n+1's); everything is
// structure-of-arrays, x fastest; walls are mirrored indices.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "lr.h"
#include "lr_device.hpp"

using namespace lr;

namespace {

template <typename GridT, typename R>
__device__ __forceinline__ bool present(const GridT &g, R V) {
  return double(V) > g.k_eps * g.A;
}

// Equation of state of material m: the perfect gas of §5.1 (pinf = 0) or
// the stiffened gas of §5.2, p = (gamma - 1) rho e - pi.  eos_krc2 is the
// material's share k rho c^2 of the mixture's bulk modulus, with the squared
// sound speed (dp/drho at constant entropy) c^2 = (gamma p + pi) / rho.
template <typename GridT, typename R>
__device__ __forceinline__ R eos_p(const GridT &g, int m, R rho, R e) {
  return R(g.gamma[m] - 1.0) * rho * e - R(g.pinf[m]);
}
template <typename GridT, typename R>
__device__ __forceinline__ R eos_krc2(const GridT &g, int m, R k, R P) {
  return k * R(g.gamma[m]) * P + k * R(g.pinf[m]);
}

// compensated accumulation for the FP32 cell totals: each addition's exact
// rounding error, the Kahan–Neumaier correction, is formed branch-free by
// Knuth's two-sum (the same error, so the same bits, one instruction fewer
// than choosing the Fast2Sum order by magnitude); needs contraction off
template <typename R>
struct Acc {
  R s, c;
  __device__ __forceinline__ void init(R v) { s = v; c = R(0); }
  __device__ __forceinline__ void add(R v) {
    const R t = s + v;
    const R bv = t - s;
    c += (s - (t - bv)) + (v - bv);
    s = t;
  }
  __device__ __forceinline__ R get() const { return s + c; }
};
template <>
struct Acc<double> {
  double s;
  __device__ __forceinline__ void init(double v) { s = v; }
  __device__ __forceinline__ void add(double v) { s += v; }
  __device__ __forceinline__ double get() const { return s; }
};

// =========================================================== mixed cells
// Partial volumes of outflow region s of mixed donor (i,j) (§4.4), FP64, one
// lane per region of a group of eight consecutive lanes: Youngs normal of the
// volume fractions, interface offset on the rectangle through the midpoints of
// the Lagrangian faces, intersection with the region's rectangle, then the
// donor-side clipping (group sums by shuffles).  d*: node displacements in the
// bulk precision, exactly as the remap kernel forms them.
template <typename R, int NM, typename ProbT>
__device__ void mixed_region_partials(const ProbT &P, const R *Vs, int i, int j, int s, R blx_r,
                                      R bly_r, R brx_r, R bry_r, R tlx_r, R tly_r, R trx_r,
                                      R try_r, R *Wout) {
  const auto &g = P.g;
  const int nx = g.nx, ny = g.ny, C = nx * ny, q = j * nx + i;
  // all of the cell's loads first (one memory latency): its partial volumes
  // and the 3x3 neighbourhood of material min(s, NM-1) for the Youngs gradient
  // formed on lane s < NM (the other lanes repeat the last material's loads)
  R Vr[NM], kr[3][3];
#pragma unroll
  for (int m = 0; m < NM; ++m) Vr[m] = ldg(Vs + (m * C + q));
  {
    const int ms = s < NM ? s : NM - 1;
#pragma unroll
    for (int bb = -1; bb <= 1; ++bb)
#pragma unroll
      for (int aa = -1; aa <= 1; ++aa)
        kr[bb + 1][aa + 1] = ldg(Vs + (ms * C + refl_cell(j + bb, ny) * nx + refl_cell(i + aa, nx)));
  }
  CellRegions<R> rr;
  cell_regions<R>(R(g.dx), R(g.dy), blx_r, bly_r, brx_r, bry_r, tlx_r, tly_r, trx_r, try_r, rr);
  R vcf_r = R(g.A);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (rr.role[k] > 0) vcf_r += rr.vol[k];
    else if (rr.role[k] < 0) vcf_r -= rr.vol[k];
  }
  const double vcf = double(vcf_r);
  const double blx = blx_r, bly = bly_r, brx = brx_r, bry = bry_r;
  const double tlx = tlx_r, tly = tly_r, trx = trx_r, try_ = try_r;
  const double hx = 0.5 * g.dx, hy = 0.5 * g.dy;
  // this lane's region (selected with static indices: no private-array
  // indexing by the lane number), its rectangle relative to the cell centre
  double fw = 0.0, ft0 = 0.0, fh = 0.0, vol = 0.0;
  bool out = false;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k == s) {
      vol = double(rr.vol[k]);
      out = rr.role[k] > 0;
      if (k < 4) {
        fw = double(rr.fg[k].w);
        ft0 = double(rr.fg[k].t0);
        fh = double(rr.fg[k].h);
      }
    }
  double x0, x1, y0, y1;
  if (s < 4) {
    const double w = fw, t0 = ft0, h = fh;
    if (s < 2) {
      const double xf = s == 0 ? -hx : hx;
      x0 = xf + fmin(0.0, w);
      x1 = xf + fmax(0.0, w);
      y0 = t0 + (-hy);
      y1 = (t0 + h) + (-hy);
    } else {
      const double yf = s == 2 ? -hy : hy;
      y0 = yf + fmin(0.0, w);
      y1 = yf + fmax(0.0, w);
      x0 = t0 + (-hx);
      x1 = (t0 + h) + (-hx);
    }
  } else {
    const double ndx = s == 4 ? blx : (s == 5 ? brx : (s == 6 ? tlx : trx));
    const double ndy = s == 4 ? bly : (s == 5 ? bry : (s == 6 ? tly : try_));
    const double cx = (s == 4 || s == 6) ? -hx : hx, cy = s < 6 ? -hy : hy;
    x0 = cx + fmin(0.0, ndx);
    x1 = cx + fmax(0.0, ndx);
    y0 = cy + fmin(0.0, ndy);
    y1 = cy + fmax(0.0, ndy);
  }
  double V[NM], Vp = 0.0;
  bool pr[NM];
  int np = 0;
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    V[m] = double(Vr[m]);
    pr[m] = V[m] > g.k_eps * g.A;
    if (pr[m]) {
      ++np;
      Vp += V[m];
    }
  }
  double W[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) W[m] = 0.0;
  const double Rx0 = 0.5 * (blx + tlx) - hx, Rx1 = 0.5 * (brx + trx) + hx;
  const double Ry0 = 0.5 * (bly + bry) - hy, Ry1 = 0.5 * (tly + try_) + hy;
  const double gmin = 1e-10 / fmin(g.dx, g.dy);
  // The per-material work of the cell is spread over its eight lanes: lane s
  // (s < NM) forms the Youngs gradient of material s, then the interface of
  // material s (for two materials, the interface of the first one present,
  // on its lane only); the other lanes read both with shuffles.  Every value
  // is formed with the same operations as on a single lane.
  static_assert(NM <= 8, "one lane of the group per material");
  const int grp = __lane_id() & ~7;
  // this lane's material's gradient (formed on every lane, used from lanes
  // s < NM: the group runs the same instructions either way)
  // (the volume fractions V/A share the cell area: the stencil takes the
  // volumes and one quotient divides by A)
  double gxs, gys;
  {
    double k[3][3];
#pragma unroll
    for (int bb = 0; bb < 3; ++bb)
#pragma unroll
      for (int aa = 0; aa < 3; ++aa) k[bb][aa] = double(kr[bb][aa]);
    gxs = ((k[0][2] + 2.0 * k[1][2] + k[2][2]) - (k[0][0] + 2.0 * k[1][0] + k[2][0])) / (8.0 * g.dx * g.A);
    gys = ((k[2][0] + 2.0 * k[2][1] + k[2][2]) - (k[0][0] + 2.0 * k[0][1] + k[0][2])) / (8.0 * g.dy * g.A);
  }
  int a0 = -1, b0 = -1;
#pragma unroll
  for (int m = 0; m < NM; ++m)
    if (pr[m]) {
      if (a0 < 0) a0 = m;
      else if (b0 < 0) b0 = m;
    }
  double GX[NM], GY[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    GX[m] = __shfl(gxs, grp + m, 64);
    GY[m] = __shfl(gys, grp + m, 64);
  }
  // interface of this lane's material: unit normal and offset, or degenerate
  double inx = 0.0, iny = 0.0, ioff = 0.0;
  int ideg = 1;
  if (s < NM && np >= 2 && pr[s] && (np > 2 || s == a0)) {
    double gx = gxs, gy = gys, Vm = 0.0;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      if (m == s) Vm = V[m];
      if (np == 2 && m == b0) {  // two materials: the difference of their gradients
        gx = gxs - GX[m];
        gy = gys - GY[m];
      }
    }
    const double nrm = sqrt(gx * gx + gy * gy);
    if (!(nrm <= gmin)) {
      inx = gx / nrm;
      iny = gy / nrm;
      ioff = interface_offset(Rx0, Rx1, Ry0, Ry1, inx, iny, Vm / Vp);
      ideg = 0;
    }
  }
  double NX[NM], NY[NM], OF[NM];
  int DG[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    NX[m] = __shfl(inx, grp + m, 64);
    NY[m] = __shfl(iny, grp + m, 64);
    OF[m] = __shfl(ioff, grp + m, 64);
    DG[m] = __shfl(ideg, grp + m, 64);
  }
  if (np == 2) {
    if (out && vol != 0.0) {
      bool deg = false;
      double nxa = 0.0, nya = 0.0, sa = 0.0;
#pragma unroll
      for (int m = 0; m < NM; ++m)
        if (m == a0) {
          deg = DG[m] != 0;
          nxa = NX[m];
          nya = NY[m];
          sa = OF[m];
        }
      if (deg) {
#pragma unroll
        for (int m = 0; m < NM; ++m)
          if (pr[m]) W[m] = vol * (V[m] / Vp);
      } else {
        double wa = rect_halfplane_area(x0, x1, y0, y1, nxa, nya, sa);
        wa = fmin(fmax(wa, 0.0), vol);
#pragma unroll
        for (int m = 0; m < NM; ++m) {
          if (m == a0) W[m] = wa;
          if (m == b0) W[m] = vol - wa;
        }
      }
    }
  } else if (np > 2) {
    bool degenerate = false;
    double raw[NM], sum = 0.0;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      // formed for every material, then kept or not: straight-line code, so
      // that the materials' areas are computed side by side
      const double ar = rect_halfplane_area(x0, x1, y0, y1, NX[m], NY[m], OF[m]);
      raw[m] = pr[m] && !DG[m] ? ar : 0.0;
      if (pr[m] && DG[m]) degenerate = true;
    }
    if (out && vol != 0.0) {
#pragma unroll
      for (int m = 0; m < NM; ++m) sum += raw[m];
#pragma unroll
      for (int m = 0; m < NM; ++m)
        if (pr[m]) W[m] = (!degenerate && sum > 0.0) ? vol * (raw[m] / sum) : vol * (V[m] / Vp);
    }
  }
  // donor-side clipping: outflow totals per material over the eight lanes
  double O[NM], Vcf[NM], room[NM], H = 0.0;
  bool over[NM], any_over = false;
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    double o = W[m];
    o += __shfl_xor(o, 1, 8);
    o += __shfl_xor(o, 2, 8);
    o += __shfl_xor(o, 4, 8);
    O[m] = o;
    Vcf[m] = (V[m] / g.A) * vcf;
    over[m] = pr[m] && O[m] > Vcf[m];
    any_over = any_over || over[m];
  }
  if (any_over) {
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      room[m] = (pr[m] && !over[m]) ? fmax(0.0, Vcf[m] - O[m]) : 0.0;
      H += room[m];
    }
    if (H > 0.0 && out) {
      double freed = 0.0;
#pragma unroll
      for (int m = 0; m < NM; ++m)
        if (over[m]) {
          const double keep = W[m] * (Vcf[m] / O[m]);
          freed += W[m] - keep;
          W[m] = keep;
        }
#pragma unroll
      for (int m = 0; m < NM; ++m)
        if (room[m] > 0.0) W[m] += freed * (room[m] / H);
    }
  }
#pragma unroll
  for (int m = 0; m < NM; ++m) stg(Wout + (s * NM + m), R(out ? W[m] : 0.0));
}

// =========================================================== k_lagrange
template <typename R, int NM, int BT, typename T>
__device__ __forceinline__ void lagrange_tile(const Prob<R> *probs, const BlockMap bm, int gpar) {
  constexpr int TX = T::TX, TY = T::TY;
  const auto &P = *cst(probs + bm.prob);
  const auto &g = P.g;
  const int par = gpar ^ P.flip;
  Slot &S = P.ctl->slot[par];
  // read with the tile's first global loads; tested once they are issued
  const bool stop = (ldg(&S.done) | ldg(&P.ctl->err)) != 0;
  const int nx = g.nx, ny = g.ny, C = nx * ny;
  const int I0 = bm.i0, J0 = bm.j0, tid = threadIdx.x;
  const R Dx = R(g.dx), Dy = R(g.dy), A = R(g.A);
  const R *Vs = P.V[par], *Ms = P.M[par], *Es = P.E[par];

  constexpr int CW = TX + 2, CH = TY + 2;  // cells [I0-1, I0+TX] x [J0-1, J0+TY]
  constexpr int NW = TX + 1, NH = TY + 1;  // nodes [I0, I0+TX] x [J0, J0+TY]
  constexpr int UW = TX + 3, UH = TY + 3;  // node velocities [I0-1, I0+TX+1] x [J0-1, J0+TY+1]
  __shared__ R sS[CH][CW], sMc[CH][CW], sQ[CH][CW];
  __shared__ R sPh[NM][CH][CW];
  __shared__ R sdx[NH][NW], sdy[NH][NW];
  __shared__ R sux[UH][UW], suy[UH][UW];
  __shared__ int s_mix[TX * TY];  // the tile's mixed cells (cell index)
  __shared__ int s_nmix, s_mixbase;

  // Global loads issued before any is used: the node velocities of the tile
  // (each once, into LDS), the cells' V, M, E (FP32, where the registers allow
  // it) and the owned cell's V, M, E (corrector).
  constexpr int NITU = (UW * UH + BT - 1) / BT;
  constexpr int NITC = (CW * CH + BT - 1) / BT;
  constexpr bool PREC = sizeof(R) == 4;
  R preu[NITU][2];
#pragma unroll
  for (int it = 0; it < NITU; ++it) {
    const int l = tid + it * BT;
    const int I = I0 - 1 + l % UW, J = J0 - 1 + l / UW;
    const bool ok = l < UW * UH && I >= 0 && J >= 0 && I <= nx && J <= ny;
    preu[it][0] = ok ? ldg(P.ux + (J * (nx + 1) + I)) : R(0);
    preu[it][1] = ok ? ldg(P.uy + (J * (nx + 1) + I)) : R(0);
  }
  // V, M, E of stage-1 cell l (the real cell it mirrors)
  auto fetchc = [&](int l, R *out) {
    const int i = I0 - 1 + l % CW, j = J0 - 1 + l / CW;
    if (l >= CW * CH || i > nx || j > ny) {
#pragma unroll
      for (int k = 0; k < 3 * NM; ++k) out[k] = R(0);
      return;
    }
    const int q = refl_cell(j, ny) * nx + refl_cell(i, nx);
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      out[m] = ldg(Vs + (m * C + q));
      out[NM + m] = ldg(Ms + (m * C + q));
      out[2 * NM + m] = ldg(Es + (m * C + q));
    }
  };
  R prec[PREC ? NITC : 1][3 * NM];
  if constexpr (PREC) {
#pragma unroll
    for (int it = 0; it < NITC; ++it) fetchc(tid + it * BT, prec[it]);
  }
  const int a3 = tid % TX, b3 = tid / TX, i3 = I0 + a3, j3 = J0 + b3;
  const bool own3 = tid < TX * TY && i3 < nx && j3 < ny;  // (BT may exceed the tile)
  const int q3 = own3 ? j3 * nx + i3 : 0;
  R pre3[3 * NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    pre3[m] = own3 ? ldg(Vs + (m * C + q3)) : R(0);
    pre3[NM + m] = own3 ? ldg(Ms + (m * C + q3)) : R(0);
    pre3[2 * NM + m] = own3 ? ldg(Es + (m * C + q3)) : R(0);
  }
  bool last;
  const R dt = R(slot_dt(g, S, last));
  if (stop) return;

#pragma unroll
  for (int it = 0; it < NITU; ++it) {
    const int l = tid + it * BT;
    if (l >= UW * UH) continue;
    sux[l / UW][l % UW] = preu[it][0];
    suy[l / UW][l % UW] = preu[it][1];
  }
  if (tid == 0) s_nmix = 0;
  __syncthreads();
  // velocity of node (I, J) of the staged window
  auto ux_at = [&](int I, int J) { return sux[J - (J0 - 1)][I - (I0 - 1)]; };
  auto uy_at = [&](int I, int J) { return suy[J - (J0 - 1)][I - (I0 - 1)]; };

  // ---- stage 1: predictor per cell (ghost cells mirror the real ones)
#pragma unroll
  for (int it = 0; it < NITC; ++it) {
    const int l = tid + it * BT;
    if (l >= CW * CH) continue;
    const int a = l % CW, b = l / CW;
    const int i = I0 - 1 + a, j = J0 - 1 + b;
    const bool owned = i >= I0 && j >= J0 && i < nx && j < ny && a <= TX && b <= TY;
    int np = 0;
    if (i <= nx && j <= ny) {
      const int ri = refl_cell(i, nx), rj = refl_cell(j, ny), q = rj * nx + ri;
      R vme[3 * NM];
      if constexpr (PREC) {
#pragma unroll
        for (int k = 0; k < 3 * NM; ++k) vme[k] = prec[it][k];
      } else {
        fetchc(l, vme);
      }
      R Msum = R(0), rc2 = R(0), k[NM], e[NM], rho[NM], Pa[NM], Mm[NM];
      bool pr[NM];
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        const R V = vme[m], M = vme[NM + m], E = vme[2 * NM + m];
        Mm[m] = M;
        k[m] = qdiv(V, A);
        pr[m] = present(g, V);
        np += pr[m];
        // an absent material's mass can be a float denormal: IEEE quotient
        e[m] = M > R(0) ? E / M : R(0);
        rho[m] = pr[m] ? qdiv(M, V) : R(0);
        Pa[m] = pr[m] ? eos_p(g, m, rho[m], e[m]) : R(0);
        if (pr[m]) rc2 += eos_krc2(g, m, k[m], Pa[m]);
        Msum += M;
      }
      R Qc = R(0), Sc = R(0);
      if (!g.kinematic) {
        const R rhoc = qdiv(Msum, A);
        const R c2 = rhoc > R(0) ? qdiv(rc2, rhoc) : R(0);
        const R cc = c2 > R(0) ? sqrt(c2) : R(0);
        const R uxbl = ux_at(ri, rj), uxbr = ux_at(ri + 1, rj), uxtl = ux_at(ri, rj + 1),
                uxtr = ux_at(ri + 1, rj + 1);
        const R uybl = uy_at(ri, rj), uybr = uy_at(ri + 1, rj), uytl = uy_at(ri, rj + 1),
                uytr = uy_at(ri + 1, rj + 1);
        const R div = qdiv(uxbr + uxtr - uxbl - uxtl, R(2) * Dx) + qdiv(uytl + uytr - uybl - uybr, R(2) * Dy);
        const R L = sqrt(A);
        if (div < R(0)) Qc = rhoc * (R(g.a1) * L * cc * fabs(div) + R(g.a2) * L * L * div * div);
        const R h = R(0.5) * dt;
        const R hblx = h * uxbl, hbly = h * uybl, hbrx = h * uxbr, hbry = h * uybr;
        const R htlx = h * uxtl, htly = h * uytl, htrx = h * uxtr, htry = h * uytr;
        R Pch = R(0);
        if constexpr (sizeof(R) == 8) {
          const R Vh = quad_area(hblx, hbly, Dx + hbrx, hbry, htlx, Dy + htly, Dx + htrx, Dy + htry);
#pragma unroll
          for (int m = 0; m < NM; ++m) {
            R Ph = R(0);
            if (pr[m]) {
              const R rho_h = Mm[m] / (k[m] * Vh);
              const R e_h = e[m] - (Pa[m] + Qc) * (R(1) / rho_h - R(1) / rho[m]);
              Ph = eos_p(g, m, rho_h, e_h);
              Pch += k[m] * Ph;
            }
            sPh[m][b][a] = Ph;
          }
        } else {
          // FP32: 1/rho^{n+1/2} - 1/rho^n = k (Vol^{n+1/2} - A) / m, with the
          // volume change from its polynomial in the displacements
          const R dV = quad_area_change(Dx, Dy, hblx, hbly, hbrx, hbry, htlx, htly, htrx, htry);
#pragma unroll
          for (int m = 0; m < NM; ++m) {
            R Ph = R(0);
            if (pr[m]) {
              const R e_h = e[m] - (Pa[m] + Qc) * qdiv(k[m] * dV, Mm[m]);
              const R rho_h = qdiv(Mm[m], k[m] * (A + dV));
              Ph = eos_p(g, m, rho_h, e_h);
              Pch += k[m] * Ph;
            }
            sPh[m][b][a] = Ph;
          }
        }
        Sc = Pch + Qc;
      }
      sS[b][a] = Sc;
      sMc[b][a] = Msum;
      sQ[b][a] = Qc;
      if (owned) {
        if (P.dbg.Q) stg(P.dbg.Q + q, Qc);
        if (P.dbg.S) stg(P.dbg.S + q, Sc);
        if (P.dbg.Ph)
          for (int m = 0; m < NM; ++m) stg(P.dbg.Ph + (m * C + q), g.kinematic ? R(0) : sPh[m][b][a]);
      }
    }
    if (owned && np >= 2) s_mix[atomicAdd(&s_nmix, 1)] = j * nx + i;
    else if (owned) stg(P.mix_slot + (j * nx + i), -1);
  }
  __syncthreads();
  // the tile's mixed cells join the problem's compact list (their interface
  // work runs in the mixed-cell kernel, spread over the whole device)
  if (tid == 0) s_mixbase = s_nmix ? atomicAdd(&S.nmix, s_nmix) : 0;
  __syncthreads();
  for (int kk = tid; kk < s_nmix; kk += BT) {
    const int q = s_mix[kk], pos = s_mixbase + kk;
    if (pos < P.mix_cap) {
      stg(P.mix_cell + pos, q);
      stg(P.mix_slot + q, pos);
    } else {
      stg(P.mix_slot + q, -1);
      atomicOr(&P.ctl->err, ERR_MIXCAP);
    }
  }

  // ---- stage 2: nodal mass, gradient of P+Q, u^{n+1/2}, u^{lag}
  for (int l = tid; l < NW * NH; l += BT) {
    const int a = l % NW, b = l / NW;
    const int I = I0 + a, J = J0 + b;
    if (I > nx || J > ny) continue;
    const int p = J * (nx + 1) + I;
    const R mp = R(0.25) * (sMc[b][a] + sMc[b][a + 1] + sMc[b + 1][a] + sMc[b + 1][a + 1]);
    R uhx, uhy, uLx, uLy;
    const R ux = ux_at(I, J), uy = uy_at(I, J);
    if (g.kinematic) {
      uhx = uLx = ux;
      uhy = uLy = uy;
    } else {
      const R sSW = sS[b][a], sSE = sS[b][a + 1], sNW = sS[b + 1][a], sNE = sS[b + 1][a + 1];
      const R gx = qdiv((sSE + sNE) - (sSW + sNW), R(2) * Dx);
      const R gy = qdiv((sNW + sNE) - (sSW + sSE), R(2) * Dy);
      const R rho_p = qdiv(mp, A);
      uhx = ux - qdiv(R(0.5) * dt * gx, rho_p);
      uhy = uy - qdiv(R(0.5) * dt * gy, rho_p);
      if (I == 0 || I == nx) uhx = R(0);
      if (J == 0 || J == ny) uhy = R(0);
      uLx = R(2) * uhx - ux;
      uLy = R(2) * uhy - uy;
      if (I == 0 || I == nx) uLx = R(0);
      if (J == 0 || J == ny) uLy = R(0);
    }
    sdx[b][a] = dt * uhx;
    sdy[b][a] = dt * uhy;
    // the tile owns nodes [I0, I0+TX) x [J0, J0+TY) (it runs over the cell
    // tiles), the last tile of a row or column also the boundary nodes
    if ((a < TX || I == nx) && (b < TY || J == ny)) {
      stg(P.uhx + p, uhx);
      stg(P.uhy + p, uhy);
      stg(P.uLx + p, uLx);
      stg(P.uLy + p, uLy);
      stg(P.mp + p, mp);
    }
  }
  __syncthreads();

  // ---- stage 3: corrector energies of the tile's cells
  {
    const int a = tid % TX, b = tid / TX;
    const int i = I0 + a, j = J0 + b;
    if (tid < TX * TY && i < nx && j < ny) {
      const int q = j * nx + i;
      const R blx = sdx[b][a], bly = sdy[b][a], brx = sdx[b][a + 1], bry = sdy[b][a + 1];
      const R tlx = sdx[b + 1][a], tly = sdy[b + 1][a], trx = sdx[b + 1][a + 1],
              try_ = sdy[b + 1][a + 1];
      const R Qc = sQ[b + 1][a + 1];
      R VL = R(0), dVL = R(0);
      if constexpr (sizeof(R) == 8) VL = quad_area(blx, bly, Dx + brx, bry, tlx, Dy + tly, Dx + trx, Dy + try_);
      else dVL = quad_area_change(Dx, Dy, blx, bly, brx, bry, tlx, tly, trx, try_);
      if (P.dbg.VL) stg(P.dbg.VL + q, sizeof(R) == 8 ? VL : A + dVL);
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        const R V = pre3[m], M = pre3[NM + m], E = pre3[2 * NM + m];
        const R e = M > R(0) ? E / M : R(0);  // M may be a denormal trace: IEEE quotient
        R eL = e;
        if (!g.kinematic && present(g, V)) {
          const R k = qdiv(V, A);
          const R Ph = sPh[m][b + 1][a + 1];
          if constexpr (sizeof(R) == 8) {
            const R rho = M / V, rhoL = M / (k * VL);
            eL = e - (Ph + Qc) * (R(1) / rhoL - R(1) / rho);
          } else {
            eL = e - (Ph + Qc) * qdiv(k * dVL, M);
          }
        }
        stg(P.eL + (m * C + q), eL);
      }
    }
  }
}

// one block per tile of the map (LOOP false: grid = map), or a grid smaller
// than the map whose blocks walk it (LOOP true; a separate instantiation,
// since the loop keeps values live across tiles and costs registers)
// WIDE: two threads per cell of the tile, for small FP64 launches (as the
// dual kernel)
template <typename R, int NM, bool LOOP, bool WIDE, typename T>
__global__ void __launch_bounds__(WIDE ? 2 * T::NT : T::NT)
    k_lagrange(const Prob<R> *probs, const BlockMap *map, int nmap, int gpar) {
  constexpr int BT = WIDE ? 2 * T::NT : T::NT;
  if constexpr (LOOP) {
    for (int b = blockIdx.x; b < nmap; b += gridDim.x) {
      lagrange_tile<R, NM, BT, T>(probs, map_entry(map, b), gpar);
      __syncthreads();  // the next tile reuses the LDS
    }
  } else {
    if (blockIdx.x < nmap) lagrange_tile<R, NM, BT, T>(probs, map_entry(map, xcd_tile(blockIdx.x, nmap)), gpar);
  }
}

// =========================================================== k_mixed
// VOF partial volumes of the mixed cells (§4.4), FP64, eight lanes per cell
// (one per flux region of the cell).  Block (x, y) takes problem plist[y]'s
// compact list of mixed cells (built by the Lagrange kernel) from entry
// 32x on, strided by 32 gridDim.x: the interface work of a problem is spread
// over the whole device instead of the tiles that hold its interfaces.  The
// node displacements are re-formed from the stored u^{n+1/2}.  Separate from
// the Lagrange kernel, whose occupancy the FP64 interface arithmetic would
// halve.
template <typename R, int NM>
__global__ void __launch_bounds__(NTHREADS) k_mixed(const Prob<R> *probs, const int *plist, int gpar) {
  const auto &P = *cst(probs + *cst(plist + blockIdx.y));
  const auto &g = P.g;
  const int par = gpar ^ P.flip;
  Slot &S = P.ctl->slot[par];
  // the stop flags, the list length, the step and the block's first list
  // entry are read together (the entry speculatively, within the list's
  // capacity)
  const bool stop = (ldg(&S.done) | ldg(&P.ctl->err)) != 0;
  const int nmix = min(ldg(&S.nmix), P.mix_cap);
  const int nx = g.nx, tid = threadIdx.x;
  const int w0 = blockIdx.x * (NTHREADS / 8) + tid / 8;
  const int q0 = ldg(P.mix_cell + min(w0, P.mix_cap - 1));
  bool last;
  const R dt = R(slot_dt(g, S, last));
  // keeps the entry's load ahead of the test (it would otherwise be sunk
  // below it, one more memory latency)
  asm volatile("" ::"v"(q0));
  if (stop || (int)blockIdx.x * (NTHREADS / 8) >= nmix) return;
  const R *Vs = P.V[par];
  for (int w = w0; w < nmix; w += gridDim.x * (NTHREADS / 8)) {
    const int q = w == w0 ? q0 : ldg(P.mix_cell + w), i = q % nx, j = q / nx;
    const int bl = j * (nx + 1) + i, br = bl + 1, tl = bl + nx + 1, tr = tl + 1;
    mixed_region_partials<R, NM>(P, Vs, i, j, tid % 8, dt * ldg(P.uhx + bl), dt * ldg(P.uhy + bl),
                                 dt * ldg(P.uhx + br), dt * ldg(P.uhy + br), dt * ldg(P.uhx + tl),
                                 dt * ldg(P.uhy + tl), dt * ldg(P.uhx + tr), dt * ldg(P.uhy + tr),
                                 P.mix_W + (size_t)w * 8 * NM);
  }
}

// =========================================================== k_remap
// Region-centred: every flux region the tile needs is formed once.
//   P1 node displacements d = dt u^{n+1/2} (2-deep halo, mirrored)
//   P2 signed volume of every x- and y-face region (the sign bit gives the
//      donor side: clear = the donor is on the -x / -y side)
//   P3 cell records (2-deep halo): rho^{lagCF}_a (Vol^{lagCF} from the
//      region volumes), e^{lag}_a, Lagrangian centre, purity; a mixed
//      record's list position is loaded here and stored after P5
//   P4 order-2 values (rho, e) of each region whose donor is pure, in the
//      donor's frame (§2.1.1, §3.3; order 1 next to another material, §4.2)
//   P5 positivity guard per donor: its order-2 outflow mass and energy
//   P6 nine-point update of the owned cells, the fluxes formed from the
//      donor's record, the region values and, for mixed donors, the
//      partial volumes formed in FP64 (§4.4)
template <typename R, int NM, typename T>
struct RemapShared {
  static constexpr int TX = T::TX, TY = T::TY;
  static constexpr int NNX = TX + 5, NNY = TY + 5;  // nodes [i0-2, i0+TX+2]
  static constexpr int NCX = TX + 4, NCY = TY + 4;  // cell records [i0-2, i0+TX+1]
  // face volumes: x-faces [i0-2, i0+TX+2] x rows [j0-2, j0+TY+1], y-faces
  // [i0-2, i0+TX+1] x [j0-2, j0+TY+2]
  static constexpr int XW = TX + 5, XH = TY + 4, YW = TX + 4, YH = TY + 5;
  // region values for donors in [i0-1, i0+TX] x [j0-1, j0+TY]: x-faces
  // [i0-1, i0+TX+1] x [j0-1, j0+TY], y-faces [i0-1, i0+TX] x [j0-1, j0+TY+1],
  // corners at nodes [i0-1, i0+TX+1] x [j0-1, j0+TY+1]
  static constexpr int VXW = TX + 3, VXH = TY + 2, VYW = TX + 2, VYH = TY + 3;
  static constexpr int VCW = TX + 3, VCH = TY + 3;
  static constexpr int NV = VXW * VXH + VYW * VYH + VCW * VCH;
  R ndx[NNY][NNX], ndy[NNY][NNX];
  R xv[XH][XW], yv[YH][YW];
  R xc[NCY][NCX], yc[NCY][NCX];
  signed char pure[NCY][NCX];  // material of a pure cell, -1 mixed; +16 once P5 keeps order 2
  // for the donors [i0-1, i0+TX] x [j0-1, j0+TY]: a pure cell's mass of its
  // material (positivity guard, P5); once P5 is done, a mixed cell's position
  // in the list of partial volumes (P6)
  union MassOrSlot {
    R mass;
    int slot;
  } mps[TY + 2][TX + 2];
  R rcf[NM][NCY][NCX], el[NM][NCY][NCX];
  // FP64: Vol^{lagCF} of the owned cells (P3 for P6); FP32 keeps it in a
  // register (the owned cell's record is its thread's first, see P3)
  R vcfo[sizeof(R) == 8 ? TY : 1][TX];
  // per region (x-faces, then y-faces, then corners): the order-2 mass and
  // energy fluxes of a pure donor in the window (set for those regions only)
  R vm[NV], vq[NV];
};

// the donor-frame region s (W, E, S, N, BL, BR, TL, TR) of region `kind`
// (0 x-face, 1 y-face, 2 corner) at (I, J), its donor cell and its index in
// the region-value arrays; `neg` is the sign bit of the signed volume (faces)
// or of the node's x-displacement (corners)
struct RegionRef {
  int di, dj, s;
};
__device__ __forceinline__ RegionRef region_donor(int kind, int I, int J, bool neg, bool mainc) {
  if (kind == 0) return neg ? RegionRef{I, J, 0} : RegionRef{I - 1, J, 1};
  if (kind == 1) return neg ? RegionRef{I, J, 2} : RegionRef{I, J - 1, 3};
  if (mainc) return neg ? RegionRef{I, J, 4} : RegionRef{I - 1, J - 1, 7};
  return neg ? RegionRef{I, J - 1, 6} : RegionRef{I - 1, J, 5};
}

template <typename R, int NM, bool REST, typename T>
__device__ __forceinline__ void remap_tile(const Prob<R> *probs, const BlockMap bm, int gpar) {
  constexpr int TX = T::TX, TY = T::TY, NT = T::NT;
  using SH = RemapShared<R, NM, T>;
  __shared__ SH sh;
  const auto &P = *cst(probs + bm.prob);
  const auto &g = P.g;
  Ctl *ctl = P.ctl;
  const int par = gpar ^ P.flip;
  const Slot &S = ctl->slot[par];
  const int i0 = bm.i0, j0 = bm.j0, tid = threadIdx.x;
  // read with the tile's first global loads; tested once they are issued
  const bool stop = (ldg(&S.done) | ldg(&ctl->err)) != 0;
  const int nx = g.nx, ny = g.ny, C = nx * ny;
  const R Dx = R(g.dx), Dy = R(g.dy), A = R(g.A);
  const R *Vs = P.V[par], *Ms = P.M[par];
  R *Vd = P.V[par ^ 1], *Md = P.M[par ^ 1], *Ed = P.E[par ^ 1];

  // Global loads issued before any is used (one memory latency for several
  // phases): u^{n+1/2} of the staged nodes (P1), the owned cell's V, M (P6)
  // and the records' V, M, e^{lag} and list positions (P3).
  constexpr int NIT1 = (SH::NNX * SH::NNY + NT - 1) / NT;
  // P3's records.  FP32: first the one of the thread's own cell (its
  // Vol^{lagCF} then stays in a register until P6, and the tile's LDS fits
  // one more block per CU), then the ring of the two-deep halo.  FP64 (two
  // blocks per CU whatever the LDS saved): in row order, which keeps every
  // wave's loads of the records in few rows.
  constexpr bool OWN_FIRST = sizeof(R) == 4;
  constexpr int NRING = SH::NCX * SH::NCY - TX * TY;
  constexpr int NIT3 = OWN_FIRST ? 1 + (NRING + NT - 1) / NT : (SH::NCX * SH::NCY + NT - 1) / NT;
  auto rec = [&](int it) {
    if constexpr (!OWN_FIRST) {
      const int l = tid + it * NT;
      return l < SH::NCX * SH::NCY ? l : -1;
    }
    if (it == 0) return (tid / TX + 2) * SH::NCX + tid % TX + 2;
    const int k = tid + (it - 1) * NT;
    if (k >= NRING) return -1;
    if (k < 2 * SH::NCX) return k;                                       // rows j0-2, j0-1
    if (k < 4 * SH::NCX) return (TY + 2) * SH::NCX + (k - 2 * SH::NCX);  // rows j0+TY, j0+TY+1
    const int r = k - 4 * SH::NCX, c = r & 3;  // two records each side of rows j0 .. j0+TY-1
    return (2 + (r >> 2)) * SH::NCX + (c < 2 ? c : TX + c);
  };
  R pre1[NIT1][2];
#pragma unroll
  for (int it = 0; it < NIT1; ++it) {
    pre1[it][0] = pre1[it][1] = R(0);
    const int l = tid + it * NT;
    if (l >= SH::NNX * SH::NNY) continue;
    const int I = i0 - 2 + l % SH::NNX, J = j0 - 2 + l / SH::NNX;
    if (I > nx + 2 || J > ny + 2) continue;
    const int p = refl_node(J, ny) * (nx + 1) + refl_node(I, nx);
    pre1[it][0] = ldg(P.uhx + p);
    pre1[it][1] = ldg(P.uhy + p);
  }
  const int a6 = tid % TX, b6 = tid / TX, i6 = i0 + a6, j6 = j0 + b6;
  const bool own6 = i6 < nx && j6 < ny;
  const int q6 = own6 ? j6 * nx + i6 : 0;
  R V6[NM], M6[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    V6[m] = own6 ? ldg(Vs + (m * C + q6)) : R(0);
    M6[m] = own6 ? ldg(Ms + (m * C + q6)) : R(0);
  }
  // V, M, e^{lag} of record l (the real cell it mirrors); loaded here in
  // FP32 launches without the at-rest skips, else in P3: in FP64 issuing them
  // early does not pay (the block is held to two per CU by its LDS and hides
  // the latency with the other), and with the skips a tile at rest reads none
  constexpr bool PRE3 = sizeof(R) == 4 && !REST;
  auto fetch3 = [&](int l, R *out) {
    const int i = i0 - 2 + l % SH::NCX, j = j0 - 2 + l / SH::NCX;
    if (l < 0 || i > nx + 1 || j > ny + 1) return;
    const int q = refl_cell(j, ny) * nx + refl_cell(i, nx);
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      out[m] = ldg(Vs + (m * C + q));
      out[NM + m] = ldg(Ms + (m * C + q));
      out[2 * NM + m] = ldg(P.eL + (m * C + q));
    }
  };
  R pre3[PRE3 ? NIT3 : 1][3 * NM];
  if constexpr (PRE3) {
#pragma unroll
    for (int it = 0; it < NIT3; ++it) fetch3(rec(it), pre3[it]);
  }
  bool last;
  const double dtd = slot_dt(g, S, last);
  const R dt = R(dtd);
  if (stop) {
    // keep the other slot stopped too, so that later launches also return
    if (i0 == 0 && j0 == 0 && tid == 0) stg(&ctl->slot[par ^ 1].done, 1);
    return;
  }

  // the first tile of the problem prepares the next step's slot (its first
  // wave clears the CFL partials)
  if (i0 == 0 && j0 == 0 && tid < 64) {
    Slot &N = ctl->slot[par ^ 1];
#pragma unroll
    for (int k = 0; k < NDT / 64; ++k)
      if (tid + 64 * k < g.ndt) stg(&N.dtmin[tid + 64 * k], (unsigned long long)__double_as_longlong(INFINITY));
    if (tid == 0) {
      const long long step = ldg(&S.step) + 1, limit = ldg(&S.limit);
      const double t = ldg(&S.t), t_end = ldg(&S.t_end);
      stg(&N.t, last ? t_end : t + dtd);
      stg(&N.t_end, t_end);
      stg(&N.step, step);
      stg(&N.limit, limit);
      stg(&N.nmix, 0);
      stg(&N.done, (last || step >= limit) ? 1 : 0);
      if (!(dtd > 0.0) || !isfinite(dtd)) atomicOr(&ctl->err, ERR_DT);
    }
  }

  // local indices: nodes and x-faces from (i0-2, j0-2), records likewise
  auto NA = [&](int I) { return I - (i0 - 2); };
  auto NB = [&](int J) { return J - (j0 - 2); };

  // ---- P1: node displacements d = dt u^{n+1/2}, mirrored at walls
#pragma unroll
  for (int it = 0; it < NIT1; ++it) {
    const int l = tid + it * NT;
    if (l >= SH::NNX * SH::NNY) continue;
    const int a = l % SH::NNX, b = l / SH::NNX;
    const int I = i0 - 2 + a, J = j0 - 2 + b;
    if (I > nx + 2 || J > ny + 2) continue;
    R dx = dt * pre1[it][0], dy = dt * pre1[it][1];
    if (refl_node(I, nx) != I) dx = -dx;
    if (refl_node(J, ny) != J) dy = -dy;
    sh.ndx[b][a] = dx;
    sh.ndy[b][a] = dy;
  }
  // A tile whose cells all have their four nodes at rest (REST launches)
  // keeps every cell's V, M and E: no region has volume, and P2 to P5 are
  // skipped (P6 takes Vol^{lagCF} = A and e^{lag} from memory).
  __syncthreads();  // the staged nodes are complete before anyone reads them
  bool tile_rest = false;
  if constexpr (REST) {
    int mine = 1;
    if (own6) {
      const int na = NA(i6), nb = NB(j6);
      mine = sh.ndx[nb][na] == R(0) && sh.ndy[nb][na] == R(0) && sh.ndx[nb][na + 1] == R(0) &&
             sh.ndy[nb][na + 1] == R(0) && sh.ndx[nb + 1][na] == R(0) && sh.ndy[nb + 1][na] == R(0) &&
             sh.ndx[nb + 1][na + 1] == R(0) && sh.ndy[nb + 1][na + 1] == R(0);
    }
    tile_rest = __syncthreads_and(mine) != 0;
  }

  // ---- P2: signed face volumes (real faces only: ghost records use the
  // real cell's faces)
  for (int l = tid; !tile_rest && l < SH::XW * SH::XH + SH::YW * SH::YH; l += NT) {
    if (l < SH::XW * SH::XH) {
      const int a = l % SH::XW, b = l / SH::XW;
      const int I = i0 - 2 + a, j = j0 - 2 + b;
      if (I < 0 || I > nx || j < 0 || j >= ny) continue;
      const FaceGeo<R> f = face_geo(sh.ndx[b][a], sh.ndy[b][a], sh.ndx[b + 1][a], sh.ndy[b + 1][a], Dy);
      const R v = fabs(f.w * f.h);
      sh.xv[b][a] = f.w >= R(0) ? v : -v;
    } else {
      const int k = l - SH::XW * SH::XH;
      const int a = k % SH::YW, b = k / SH::YW;
      const int i = i0 - 2 + a, J = j0 - 2 + b;
      if (i < 0 || i >= nx || J < 0 || J > ny) continue;
      const FaceGeo<R> f = face_geo(sh.ndy[b][a], sh.ndx[b][a], sh.ndy[b][a + 1], sh.ndx[b][a + 1], Dx);
      const R v = fabs(f.w * f.h);
      sh.yv[b][a] = f.w >= R(0) ? v : -v;
    }
  }
  __syncthreads();

  // Vol^{lagCF} of the real cell whose BL node is staged at (na, nb):
  // A + outflow - inflow over W, E, S, N, BL, BR, TL, TR (formed in P3 for
  // every record; P6 reads the owned cells' from LDS)
  auto cell_volcf = [&](int na, int nb) {
    R v = A;
    const R xw = sh.xv[nb][na], xe = sh.xv[nb][na + 1], ys = sh.yv[nb][na], yn = sh.yv[nb + 1][na];
    if (signbit(xw)) v += fabs(xw); else v -= fabs(xw);
    if (!signbit(xe)) v += fabs(xe); else v -= fabs(xe);
    if (signbit(ys)) v += fabs(ys); else v -= fabs(ys);
    if (!signbit(yn)) v += fabs(yn); else v -= fabs(yn);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const R cx = sh.ndx[nb + (c >> 1)][na + (c & 1)], cy = sh.ndy[nb + (c >> 1)][na + (c & 1)];
      const bool sx = cx >= R(0), sy = cy >= R(0);
      const R vol = fabs(cx * cy);
      int role;
      if (c == 0) role = (sx == sy) ? (sx ? -1 : 1) : 0;       // cell is NE of its BL node
      else if (c == 1) role = (sx != sy) ? (sx ? 1 : -1) : 0;  // NW of its BR node
      else if (c == 2) role = (sx != sy) ? (sx ? -1 : 1) : 0;  // SE of its TL node
      else role = (sx == sy) ? (sx ? 1 : -1) : 0;              // SW of its TR node
      if (role > 0) v += vol;
      else if (role < 0) v -= vol;
    }
    return v;
  };

  // ---- P3: cell records; ghost cells mirror the real ones
  int ms3[NIT3];  // list position of a mixed record (-1: not listed); -2 not mixed
  R vcf_own = A;  // Vol^{lagCF} of the thread's own cell
#pragma unroll
  for (int it = 0; it < NIT3; ++it) {
    ms3[it] = -2;
    const int l = rec(it);
    if (tile_rest || l < 0) continue;
    const int a = l % SH::NCX, b = l / SH::NCX;
    const int i = i0 - 2 + a, j = j0 - 2 + b;
    if (i > nx + 1 || j > ny + 1) continue;
    R vme[3 * NM];
    if constexpr (PRE3) {
#pragma unroll
      for (int k = 0; k < 3 * NM; ++k) vme[k] = pre3[it][k];
    } else {
      fetch3(l, vme);
    }
    const int ri = refl_cell(i, nx), rj = refl_cell(j, ny), q = rj * nx + ri;
    const int na = NA(ri), nb = NB(rj);  // local node of the real cell's BL node
    const R blx = sh.ndx[nb][na], bly = sh.ndy[nb][na], brx = sh.ndx[nb][na + 1],
            bry = sh.ndy[nb][na + 1];
    const R tlx = sh.ndx[nb + 1][na], tly = sh.ndy[nb + 1][na], trx = sh.ndx[nb + 1][na + 1],
            try_ = sh.ndy[nb + 1][na + 1];
    const R v = cell_volcf(na, nb);
    R xc = R(0.25) * ((R(ri) * Dx + blx) + (R(ri + 1) * Dx + brx) + (R(ri) * Dx + tlx) +
                      (R(ri + 1) * Dx + trx));
    R yc = R(0.25) * ((R(rj) * Dy + bly) + (R(rj) * Dy + bry) + (R(rj + 1) * Dy + tly) +
                      (R(rj + 1) * Dy + try_));
    if (ri != i) xc = (i < 0 ? R(0) : R(2.0 * g.Lx)) - xc;
    if (rj != j) yc = (j < 0 ? R(0) : R(2.0 * g.Ly)) - yc;
    sh.xc[b][a] = xc;
    sh.yc[b][a] = yc;
    if constexpr (OWN_FIRST) {
      if (it == 0) vcf_own = v;
    } else if (a >= 2 && b >= 2 && a < TX + 2 && b < TY + 2) {
      sh.vcfo[b - 2][a - 2] = v;
    }
    int np = 0, pm = -1;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const R V = vme[m], M = vme[NM + m];
      const bool pr = present(g, V);
      if (pr) {
        ++np;
        pm = m;
      }
      sh.rcf[m][b][a] = pr ? qdiv(M, qdiv(V, A) * v) : R(0);
      sh.el[m][b][a] = vme[2 * NM + m];
    }
    sh.pure[b][a] = np == 1 ? pm : -1;
    // a mixed record's list position: loaded here, stored in LDS after P5,
    // so that the load's latency is spent on P4 and P5
    const bool ring1 = a >= 1 && b >= 1 && a <= TX + 2 && b <= TY + 2;  // a donor of the tile's regions
    ms3[it] = np >= 2 && ring1 ? ldg(P.mix_slot + q) : -2;
    R mp = R(0);
#pragma unroll
    for (int m = 0; m < NM; ++m)
      if (m == pm) mp = vme[NM + m];
    if (ring1) sh.mps[b - 1][a - 1].mass = mp;
    if (ri == i && rj == j && a >= 2 && b >= 2 && a < TX + 2 && b < TY + 2) {
      if (!(v > R(0))) atomicOr(&ctl->err, ERR_VOLCF);
      if (P.dbg.volcf) stg(P.dbg.volcf + q, v);
      if (P.dbg.dxL) {  // the widths P4 forms for this cell as a donor
        stg(P.dbg.dxL + q, Dx + R(0.5) * ((brx + trx) - (blx + tlx)));
        stg(P.dbg.dyL + q, Dy + R(0.5) * ((tly + try_) - (bly + bry)));
      }
      if (P.dbg.rhocf)
        for (int m = 0; m < NM; ++m) stg(P.dbg.rhocf + (m * C + q), sh.rcf[m][b][a]);
    }
  }
  __syncthreads();

  const R nrm = sqrt(Dx * Dx + Dy * Dy);
  const R dgx = Dx / nrm, dgy = Dy / nrm;  // unit vector of the main diagonal
  // order 2: limited linear along each region's direction; order 3: the
  // multidimensional least-squares plane (§3.3); both form P4's values
  const bool o2 = g.recon_order >= 2, o3 = g.recon_order == 3;
  // in-tile window of the donors whose regions the tile needs
  auto donor_in = [&](int di, int dj) {
    return di >= i0 - 1 && di <= i0 + TX && dj >= j0 - 1 && dj <= j0 + TY && di >= 0 && dj >= 0 &&
           di < nx && dj < ny;
  };
  // region (kind, I, J) -> index in vr/ve
  auto vidx = [&](int kind, int I, int J) {
    if (kind == 0) return (J - (j0 - 1)) * SH::VXW + (I - (i0 - 1));
    if (kind == 1) return SH::VXW * SH::VXH + (J - (j0 - 1)) * SH::VYW + (I - (i0 - 1));
    return SH::VXW * SH::VXH + SH::VYW * SH::VYH + (J - (j0 - 1)) * SH::VCW + (I - (i0 - 1));
  };
  // signed volume of region (kind, I, J) (real position); for corners the
  // sign is that of the node's x-displacement and *mainc its kind
  auto region_vol = [&](int kind, int I, int J, bool &mainc) {
    mainc = false;
    if (kind == 0) return sh.xv[NB(J)][NA(I)];
    if (kind == 1) return sh.yv[NB(J)][NA(I)];
    const R cdx = sh.ndx[NB(J)][NA(I)], cdy = sh.ndy[NB(J)][NA(I)];
    mainc = corner_main(cdx, cdy);
    const R v = fabs(cdx * cdy);
    return cdx >= R(0) ? v : -v;
  };

  // ---- P4: order-2 values of the regions with a pure donor in the window
  if (o2 && !tile_rest) {
    for (int l = tid; l < SH::NV; l += NT) {
      int kind, I, J;
      if (l < SH::VXW * SH::VXH) {
        kind = 0; I = i0 - 1 + l % SH::VXW; J = j0 - 1 + l / SH::VXW;
        if (I < 0 || I > nx || J < 0 || J >= ny) continue;
      } else if (l < SH::VXW * SH::VXH + SH::VYW * SH::VYH) {
        const int k = l - SH::VXW * SH::VXH;
        kind = 1; I = i0 - 1 + k % SH::VYW; J = j0 - 1 + k / SH::VYW;
        if (I < 0 || I >= nx || J < 0 || J > ny) continue;
      } else {
        const int k = l - SH::VXW * SH::VXH - SH::VYW * SH::VYH;
        kind = 2; I = i0 - 1 + k % SH::VCW; J = j0 - 1 + k / SH::VCW;
        if (I < 0 || I > nx || J < 0 || J > ny) continue;
      }
      bool mainc;
      const R sv = region_vol(kind, I, J, mainc);
      if (REST && sv == R(0)) {  // no flow: zero fluxes, and no slopes to form
        sh.vm[l] = R(0);
        sh.vq[l] = R(0);
        continue;
      }
      const RegionRef rf = region_donor(kind, I, J, signbit(sv), mainc);
      if (!donor_in(rf.di, rf.dj)) continue;
      const int ca = rf.di - (i0 - 2), cb = rf.dj - (j0 - 2);
      const int pm = sh.pure[cb][ca];
      if (pm < 0) continue;
      // LDS indexed by the material directly (no private array is indexed)
      const R rD = sh.rcf[pm][cb][ca], eD = sh.el[pm][cb][ca];
      R vr = rD, ve = eD;
      const int na = NA(rf.di), nb = NB(rf.dj);  // donor's BL node
      // the donor's Lagrangian widths, from the nodes of the real cell it
      // mirrors (as its record's centre is formed)
      const int ra = NA(refl_cell(rf.di, nx)), rb = NB(refl_cell(rf.dj, ny));
      auto width_x = [&]() {
        return Dx + R(0.5) * ((sh.ndx[rb][ra + 1] + sh.ndx[rb + 1][ra + 1]) - (sh.ndx[rb][ra] + sh.ndx[rb + 1][ra]));
      };
      auto width_y = [&]() {
        return Dy + R(0.5) * ((sh.ndy[rb + 1][ra] + sh.ndy[rb + 1][ra + 1]) - (sh.ndy[rb][ra] + sh.ndy[rb][ra + 1]));
      };
      const int s = rf.s;
      if (o3) {
        // §3.3 multidimensional: the plane over the donor's 3 x 3 records,
        // its gradient the least-squares fit of the neighbours' values at
        // their Lagrangian centres (normal equations, cofactor inverse),
        // scaled to the smallest of the four limited directional slopes,
        // evaluated at the centre of the region's flux rectangle; order 1
        // unless all nine records are pure cells of the donor's material
        bool ok = true;
#pragma unroll
        for (int b = -1; b <= 1; ++b)
#pragma unroll
          for (int a = -1; a <= 1; ++a) ok = ok && sh.pure[cb + b][ca + a] == pm;
        if (ok) {
          const R xD = sh.xc[cb][ca], yD = sh.yc[cb][ca];
          R s11 = R(0), s12 = R(0), s22 = R(0), br1 = R(0), br2 = R(0), be1 = R(0), be2 = R(0);
          // (rolled loops: unrolled, the neighbours' loads are all hoisted
          // and their registers would set the kernel's occupancy for every
          // reconstruction order)
#pragma unroll 1
          for (int b = -1; b <= 1; ++b)
#pragma unroll 1
            for (int a = -1; a <= 1; ++a) {
              if (a == 0 && b == 0) continue;
              const R X1 = sh.xc[cb + b][ca + a] - xD, X2 = sh.yc[cb + b][ca + a] - yD;
              const R Ar = sh.rcf[pm][cb + b][ca + a] - rD, Ae = sh.el[pm][cb + b][ca + a] - eD;
              s11 += X1 * X1; s12 += X1 * X2; s22 += X2 * X2;
              br1 += X1 * Ar; br2 += X2 * Ar;
              be1 += X1 * Ae; be2 += X2 * Ae;
            }
          const R det = s11 * s22 - s12 * s12;
          // the centre of the region's flux rectangle (the frame of xc, yc)
          R xr, yr;
          if (s < 4) {
            const bool xf = s < 2;
            const int I = xf ? rf.di + (s == 1) : rf.di, J = xf ? rf.dj : rf.dj + (s == 3);
            const int a0 = NA(I), b0 = NB(J);
            const FaceGeo<R> fg = xf ? face_geo(sh.ndx[b0][a0], sh.ndy[b0][a0], sh.ndx[b0 + 1][a0], sh.ndy[b0 + 1][a0], Dy)
                                     : face_geo(sh.ndy[b0][a0], sh.ndx[b0][a0], sh.ndy[b0][a0 + 1], sh.ndx[b0][a0 + 1], Dx);
            xr = xf ? R(I) * Dx + R(0.5) * fg.w : R(I) * Dx + (fg.t0 + R(0.5) * fg.h);
            yr = xf ? R(J) * Dy + (fg.t0 + R(0.5) * fg.h) : R(J) * Dy + R(0.5) * fg.w;
          } else {
            const int cn = s - 4;
            const int a0 = na + (cn & 1), b0 = nb + (cn >> 1);
            xr = R(rf.di + (cn & 1)) * Dx + R(0.5) * sh.ndx[b0][a0];
            yr = R(rf.dj + (cn >> 1)) * Dy + R(0.5) * sh.ndy[b0][a0];
          }
          if (det > R(0)) {
            const R Gr1 = (s22 * br1 - s12 * br2) / det, Gr2 = (s11 * br2 - s12 * br1) / det;
            const R Ge1 = (s22 * be1 - s12 * be2) / det, Ge2 = (s11 * be2 - s12 * be1) / det;
            // the four limited slopes: x, y, v, v_perp
            R limr = R(INFINITY), lime = R(INFINITY);
#pragma unroll 1
            for (int dd = 0; dd < 4; ++dd) {
              const int si = dd == 1 ? 0 : 1, sj = dd == 0 ? 0 : (dd == 3 ? -1 : 1);
              const R vx = dd == 0 ? R(1) : (dd == 1 ? R(0) : dgx);
              const R vy = dd == 0 ? R(0) : (dd == 1 ? R(1) : (dd == 2 ? dgy : -dgy));
              const int am = ca - si, bmn = cb - sj, ap = ca + si, bp = cb + sj;
              const R lm = (xD - sh.xc[bmn][am]) * vx + (yD - sh.yc[bmn][am]) * vy;
              const R lp = (sh.xc[bp][ap] - xD) * vx + (sh.yc[bp][ap] - yD) * vy;
              limr = fmin(limr, fabs(van_leer_d(rD - sh.rcf[pm][bmn][am], sh.rcf[pm][bp][ap] - rD, lm, lp)));
              lime = fmin(lime, fabs(van_leer_d(eD - sh.el[pm][bmn][am], sh.el[pm][bp][ap] - eD, lm, lp)));
            }
            const R ngr = sqrt(Gr1 * Gr1 + Gr2 * Gr2), nge = sqrt(Ge1 * Ge1 + Ge2 * Ge2);
            if (ngr > R(0)) vr = rD + (limr / ngr) * (Gr1 * (xr - xD) + Gr2 * (yr - yD));
            if (nge > R(0)) ve = eD + (lime / nge) * (Ge1 * (xr - xD) + Ge2 * (yr - yD));
          }
        }
        const R mu = vr * fabs(sv);
        sh.vm[l] = mu;
        sh.vq[l] = mu * ve;
        continue;
      }
      int si, sj;
      R vx, vy, off;
      if (s < 2) {
        const R sg = s == 0 ? R(-1) : R(1);
        const R lo = sh.ndx[nb][na + (s == 1)], hi = sh.ndx[nb + 1][na + (s == 1)];
        si = 1; sj = 0; vx = R(1); vy = R(0);
        off = sg * width_x() - R(0.5) * (lo + hi);
      } else if (s < 4) {
        const R sg = s == 2 ? R(-1) : R(1);
        const R lo = sh.ndy[nb + (s == 3)][na], hi = sh.ndy[nb + (s == 3)][na + 1];
        si = 0; sj = 1; vx = R(0); vy = R(1);
        off = sg * width_y() - R(0.5) * (lo + hi);
      } else {
        const R dxL = width_x(), dyL = width_y();
        const int cn = s - 4;  // BL, BR, TL, TR node of the donor
        const R cdx = sh.ndx[nb + (cn >> 1)][na + (cn & 1)], cdy = sh.ndy[nb + (cn >> 1)][na + (cn & 1)];
        const R sx = cdx >= R(0) ? R(1) : R(-1);
        if (corner_main(cdx, cdy)) {
          si = 1; sj = 1; vx = dgx; vy = dgy;
          off = (sx * dxL - cdx) * vx + (sx * dyL - cdy) * vy;
        } else {
          si = 1; sj = -1; vx = dgx; vy = -dgy;
          off = (sx * dxL - cdx) * vx + (-sx * dyL - cdy) * vy;
        }
      }
      const int am = ca - si, bmn = cb - sj, ap = ca + si, bp = cb + sj;
      if (sh.pure[bmn][am] == pm && sh.pure[bp][ap] == pm) {
        const R xD = sh.xc[cb][ca], yD = sh.yc[cb][ca];
        const R lm = (xD - sh.xc[bmn][am]) * vx + (yD - sh.yc[bmn][am]) * vy;
        const R lp = (sh.xc[bp][ap] - xD) * vx + (sh.yc[bp][ap] - yD) * vy;
        const R rm = sh.rcf[pm][bmn][am], rp = sh.rcf[pm][bp][ap];
        const R em = sh.el[pm][bmn][am], ep = sh.el[pm][bp][ap];
        vr = rD + R(0.5) * van_leer_d(rD - rm, rp - rD, lm, lp) * off;
        ve = eD + R(0.5) * van_leer_d(eD - em, ep - eD, lm, lp) * off;
      }
      const R mu = vr * fabs(sv);
      sh.vm[l] = mu;
      sh.vq[l] = mu * ve;
    }
    __syncthreads();

    // ---- P5: positivity guard of each pure donor of the window: order 2
    // is kept unless it would send out more mass or energy than it holds
    for (int l = tid; l < (TX + 2) * (TY + 2); l += NT) {
      const int di = i0 - 1 + l % (TX + 2), dj = j0 - 1 + l / (TX + 2);
      if (di >= nx || dj >= ny || di < 0 || dj < 0) continue;
      const int ca = di - (i0 - 2), cb = dj - (j0 - 2);
      const int pm = sh.pure[cb][ca];
      if (pm < 0) continue;
      const R Mpm = sh.mps[cb - 1][ca - 1].mass;
      const R eD = sh.el[pm][cb][ca];
      // the donor's eight regions in the region arrays: W, E faces, S, N
      // faces, corners at its BL, BR, TL, TR nodes.  A region is an outflow
      // of this donor iff the donor choice of P4 (sign of the region's volume,
      // the corner's diagonal) names it
      const int vx0 = vidx(0, di, dj), vy0 = vidx(1, di, dj), vc0 = vidx(2, di, dj);
      const int vi8[8] = {vx0, vx0 + 1, vy0, vy0 + SH::VYW, vc0, vc0 + 1, vc0 + SH::VCW, vc0 + SH::VCW + 1};
      const int na = NA(di), nb = NB(dj);
      bool out[8];
      out[0] = signbit(sh.xv[nb][na]);
      out[1] = !signbit(sh.xv[nb][na + 1]);
      out[2] = signbit(sh.yv[nb][na]);
      out[3] = !signbit(sh.yv[nb + 1][na]);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const R cdx = sh.ndx[nb + (c >> 1)][na + (c & 1)], cdy = sh.ndy[nb + (c >> 1)][na + (c & 1)];
        const bool mainc = corner_main(cdx, cdy), neg = !(cdx >= R(0));
        // BL: main diagonal, flow to -x; BR: anti, +x; TL: anti, -x; TR: main, +x
        out[4 + c] = (c == 0 || c == 3) ? (mainc && neg == (c == 0)) : (!mainc && neg == (c == 2));
      }
      R Mout = R(0), Eout = R(0);
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        if (!out[s]) continue;
        const int vi = vi8[s];
        Mout += sh.vm[vi];
        Eout += sh.vq[vi];
      }
      if (!(Mout > Mpm || Eout > Mpm * eD)) sh.pure[cb][ca] = pm + 16;
    }
  }
#pragma unroll
  for (int it = 0; it < NIT3; ++it) {
    const int l = rec(it);  // (ms3 is -2 outside the donor ring)
    if (l >= 0 && ms3[it] != -2) sh.mps[l / SH::NCX - 1][l % SH::NCX - 1].slot = ms3[it];
  }
  __syncthreads();

  // ---- P6: nine-point update of the tile's cells
  {
    const int a = tid % TX, b = tid / TX;
    const int i = i0 + a, j = j0 + b;
    if (i < nx && j < ny) {
      const int q = j * nx + i;
      const int ca = a + 2, cb = b + 2;
      // V^{lagCF}_a = k_a Vol^{lagCF}, formed first (few values are live here)
      R Vcf[NM], elc[NM];
      {
        R v = A;
        if (tile_rest) {
#pragma unroll
          for (int m = 0; m < NM; ++m) elc[m] = ldg(P.eL + (m * C + q));
        } else {
          if constexpr (OWN_FIRST) v = vcf_own;
          else v = sh.vcfo[b][a];
#pragma unroll
          for (int m = 0; m < NM; ++m) elc[m] = sh.el[m][cb][ca];
        }
#pragma unroll
        for (int m = 0; m < NM; ++m) Vcf[m] = qdiv(V6[m], A) * v;
      }
      // regions W, E, S, N (faces) and the corners at BL, BR, TL, TR;
      // sign +: into this cell along the region's orientation; walls and
      // corners of the other diagonal carry nothing
      const int rk[8] = {0, 0, 1, 1, 2, 2, 2, 2};
      const int rI[8] = {i, i + 1, i, i, i, i + 1, i, i + 1};
      const int rJ[8] = {j, j, j, j + 1, j, j, j + 1, j + 1};
      // The eight regions of the cell are bounded by its own four nodes' old
      // and new positions: with those four at rest (REST launches) every
      // region has zero volume, the cell keeps V^{lagCF}, M and E, and the
      // regions are not formed (their fluxes and sums below are skipped).
      bool rest = false;
      if constexpr (REST) {
        const int na = NA(i), nb = NB(j);
        rest = sh.ndx[nb][na] == R(0) && sh.ndy[nb][na] == R(0) && sh.ndx[nb][na + 1] == R(0) &&
               sh.ndy[nb][na + 1] == R(0) && sh.ndx[nb + 1][na] == R(0) && sh.ndy[nb + 1][na] == R(0) &&
               sh.ndx[nb + 1][na + 1] == R(0) && sh.ndy[nb + 1][na + 1] == R(0);
      }
      // first every region's donor, and the loads of the partial volumes of
      // the mixed donors (all issued before any is used); then each region's
      // fluxes, added at once to the cell's sums.  Each sum takes its terms
      // in region order; a region adds only to the materials it carries (a
      // pure donor's to one), the others' terms being zero.
      R sgn[8], wr[8], dirs[8];
      int dd[8], pqs[8], mss[8];
      R wmx[8][NM];  // unset unless the region's donor is mixed
      Acc<R> Va[NM], Ma[NM], Ea[NM];
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        Va[m].init(Vcf[m]);
        Ma[m].init(M6[m]);
        Ea[m].init(M6[m] * elc[m]);
      }
      // total mass flux of the regions this cell owns (left face, bottom face,
      // bottom-left corner) for the momentum remap; walls are zero
      R mx = R(0), my = R(0), mc = R(0);
      const bool dbg_w = P.dbg.Wpx != nullptr;
      const int nX = (nx + 1) * ny, nY = nx * (ny + 1), nN = (nx + 1) * (ny + 1);
      if (dbg_w && rest)
        for (int m = 0; m < NM; ++m) {
          stg(P.dbg.Wpx + (m * nX + j * (nx + 1) + i), R(0));
          stg(P.dbg.Wpy + (m * nY + j * nx + i), R(0));
          stg(P.dbg.Wpc + (m * nN + j * (nx + 1) + i), R(0));
        }
      if (!rest) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        bool mainc;
        const R sv = region_vol(rk[s], rI[s], rJ[s], mainc);
        // the flux of the bottom-left corner (either diagonal) also goes to
        // the momentum remap, so it is formed even when this cell is not
        // one of its two cells
        bool need;
        if (s == 0) sgn[s] = i > 0 ? R(1) : R(0);
        else if (s == 1) sgn[s] = i < nx - 1 ? R(-1) : R(0);
        else if (s == 2) sgn[s] = j > 0 ? R(1) : R(0);
        else if (s == 3) sgn[s] = j < ny - 1 ? R(-1) : R(0);
        if (s < 4) {
          need = sgn[s] != R(0);
        } else {
          const int I = rI[s], J = rJ[s];
          const bool wall = I == 0 || I == nx || J == 0 || J == ny;
          const bool mine = (s == 4 || s == 7) ? mainc : !mainc;
          sgn[s] = (!wall && mine) ? ((s == 4 || s == 6) ? R(1) : R(-1)) : R(0);
          need = s == 4 ? !wall : sgn[s] != R(0);
        }
        const bool neg = signbit(sv);
        const RegionRef rf = region_donor(rk[s], rI[s], rJ[s], neg, mainc);
        dirs[s] = neg ? R(-1) : R(1);
        wr[s] = fabs(sv);
        const int da = rf.di - (i0 - 2), db = rf.dj - (j0 - 2);
        dd[s] = db * SH::NCX + da;
        pqs[s] = need ? int(sh.pure[db][da]) : -2;  // -2: no flux
        mss[s] = -1;
        if (pqs[s] == -1) {
          const int ms = sh.mps[db - 1][da - 1].slot;
          if (ms >= 0 && ms < P.mix_cap) {
            mss[s] = ms;
            const R *src = P.mix_W + (size_t)ms * 8 * NM + rf.s * NM;
#pragma unroll
            for (int m = 0; m < NM; ++m) wmx[s][m] = ldg(src + m);
          }
        }
      }
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        R F[3 * NM];  // this region's V, M, E per material, signed along its orientation
#pragma unroll
        for (int k = 0; k < 3 * NM; ++k) F[k] = R(0);
        const int pq = pqs[s], d = dd[s];  // donor record, flattened
        const R dir = dirs[s], w = wr[s];
        const R sg = sgn[s];
        if (pq >= 0) {
          const int pm = pq & 15;
          const R rho = (&sh.rcf[pm][0][0])[d], e = (&sh.el[pm][0][0])[d];
          R mu = w > R(0) ? rho * w : R(0);
          R ep = w > R(0) ? mu * e : R(0);
          if (o2 && pq >= 16) {  // order 2 kept by the guard: the region's own fluxes
            const int vi = vidx(rk[s], rI[s], rJ[s]);
            mu = w > R(0) ? sh.vm[vi] : R(0);
            ep = w > R(0) ? sh.vq[vi] : R(0);
          }
#pragma unroll
          for (int m = 0; m < NM; ++m)
            if (m == pm) {
              F[m] = dir * w;
              F[NM + m] = dir * mu;
              F[2 * NM + m] = dir * ep;
              if (sg > R(0)) { Va[m].add(F[m]); Ma[m].add(F[NM + m]); Ea[m].add(F[2 * NM + m]); }
              else if (sg < R(0)) { Va[m].add(-F[m]); Ma[m].add(-F[NM + m]); Ea[m].add(-F[2 * NM + m]); }
            }
        } else if (pq == -1 && mss[s] >= 0) {
#pragma unroll
          for (int m = 0; m < NM; ++m) {
            const R wm = wmx[s][m];
            const R mu = wm > R(0) ? (&sh.rcf[m][0][0])[d] * wm : R(0);
            const R ep = wm > R(0) ? mu * (&sh.el[m][0][0])[d] : R(0);
            F[m] = dir * wm;
            F[NM + m] = dir * mu;
            F[2 * NM + m] = dir * ep;
            if (sg > R(0)) { Va[m].add(F[m]); Ma[m].add(F[NM + m]); Ea[m].add(F[2 * NM + m]); }
            else if (sg < R(0)) { Va[m].add(-F[m]); Ma[m].add(-F[NM + m]); Ea[m].add(-F[2 * NM + m]); }
          }
        }
        if (s == 0 || s == 2 || s == 4) {
          R f = R(0);
#pragma unroll
          for (int m = 0; m < NM; ++m) f += F[NM + m];
          if (s == 0) mx = f;
          else if (s == 2) my = f;
          else mc = f;
          if (dbg_w)
            for (int m = 0; m < NM; ++m) {
              if (s == 0) stg(P.dbg.Wpx + (m * nX + j * (nx + 1) + i), i > 0 ? F[m] : R(0));
              else if (s == 2) stg(P.dbg.Wpy + (m * nY + j * nx + i), j > 0 ? F[m] : R(0));
              else stg(P.dbg.Wpc + (m * nN + j * (nx + 1) + i), (i > 0 && j > 0) ? F[m] : R(0));
            }
        }
      }
      }  // !rest
      R Vn[NM], Mn[NM], En[NM], Msa = R(0), Esa = R(0);
      bool bad_nan = false;
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        Vn[m] = Va[m].get();
        Mn[m] = Ma[m].get();
        En[m] = Ea[m].get();
        if constexpr (sizeof(R) == 4) {
          // FP32: a material below the presence threshold that the update
          // leaves with a negative volume, mass or energy is removed from the
          // cell.  Such values are rounding residues (about 1e-8 of a cell in
          // single precision); left in place, the cell's volume change
          // Vol^{lagCF}/A scales them step after step, and over hundreds of
          // steps of expansion they grow past the negativity tolerance.
          if (!present(g, Vn[m]) && (Vn[m] < R(0) || Mn[m] < R(0) || En[m] < R(0)))
            Vn[m] = Mn[m] = En[m] = R(0);
        }
        stg(Vd + (m * C + q), Vn[m]);
        stg(Md + (m * C + q), Mn[m]);
        stg(Ed + (m * C + q), En[m]);
        Msa += fabs(Mn[m]);
        Esa += fabs(En[m]);
        if (!isfinite(Vn[m]) || !isfinite(Mn[m]) || !isfinite(En[m])) bad_nan = true;
      }
      bool bad_neg = false;
      R rc2 = R(0), Msum = R(0);
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        const R tol = R(-g.neg_tol);
        if (Vn[m] < tol * A || Mn[m] < tol * Msa || En[m] < tol * Esa) bad_neg = true;
        if (present(g, Vn[m])) {
          const R rho = qdiv(Mn[m], Vn[m]);
          const R e = Mn[m] > R(0) ? qdiv(En[m], Mn[m]) : R(0);
          const R Pm = eos_p(g, m, rho, e);
          rc2 += eos_krc2(g, m, qdiv(Vn[m], A), Pm);
        }
        Msum += Mn[m];
      }
      if (bad_nan) atomicOr(&ctl->err, ERR_NAN);
      else if (bad_neg) atomicOr(&ctl->err, ERR_NEG);
      const R rhoc = qdiv(Msum, A);
      const R c2 = rhoc > R(0) ? qdiv(rc2, rhoc) : R(0);
      stg(P.cs + q, c2 > R(0) ? sqrt(c2) : R(0));
      stg(P.MX + (j * (nx + 1) + i), i > 0 ? mx : R(0));
      stg(P.MY + (j * nx + i), j > 0 ? my : R(0));
      stg(P.MC + (j * (nx + 1) + i), (i > 0 && j > 0) ? mc : R(0));
    }
  }
}

// one block per tile of the map (LOOP false: grid = map), or a grid smaller
// than the map whose blocks walk it (LOOP true; a separate instantiation,
// since the loop keeps values live across tiles and costs registers)
// REST: regions of zero volume (material at rest) skip the order-2 values.
// Launches of many tiles gain by it; a small FP64 launch, timed by its
// slowest tile, runs without the test.
template <typename R, int NM, bool LOOP, bool REST, typename T>
__global__ void __launch_bounds__(T::NT) k_remap(const Prob<R> *probs, const BlockMap *map, int nmap,
                                               int gpar) {
  if constexpr (LOOP) {
    for (int b = blockIdx.x; b < nmap; b += gridDim.x) {
      remap_tile<R, NM, REST, T>(probs, map_entry(map, b), gpar);
      __syncthreads();  // the next tile reuses the LDS
    }
  } else {
    if (blockIdx.x < nmap) remap_tile<R, NM, REST, T>(probs, map_entry(map, xcd_tile(blockIdx.x, nmap)), gpar);
  }
}

// =========================================================== k_dual
template <typename R, typename T>
struct DualShared {
  static constexpr int TX = T::TX, TY = T::TY;
  static constexpr int NX_ = TX + 4, NY_ = TY + 4;  // nodes [I0-2, I0+TX+1]
  static constexpr int NXF = (TX + 1) * TY, NYF = TX * (TY + 1), NCN = (TX + 1) * (TY + 1);
  // primal mass fluxes around the tile, mirrored at walls: x-faces
  // [I0-1, I0+TX] x rows [J0-1, J0+TY-1]; y-faces columns [I0-1, I0+TX-1] x
  // [J0-1, J0+TY]; (main, anti) corner fluxes at nodes [I0-1, I0+TX] x [J0-1, J0+TY]
  static constexpr int PXW = TX + 2, PXH = TY + 1, PYW = TX + 1, PYH = TY + 2;
  static constexpr int PCW = TX + 2, PCH = TY + 2;
  R ulx[NY_][NX_], uly[NY_][NX_];
  // node displacements (x, y) while the regions are formed; after that their
  // storage holds the anti-diagonal corners' momentum fluxes (FA)
  R dxy[2][NY_][NX_];
  R mx[PXH][PXW], my[PYH][PYW], cd[PCH][PCW], ca[PCH][PCW];
  // momentum fluxes (x, y components) of the dual regions; their mass fluxes
  // are re-formed from the staged primal fluxes where the nodes sum them
  R fx[2][NXF], fy[2][NYF], fd[2][NCN];
  static constexpr int FA = NCN;  // component c of corner k at (&dxy[0][0][0])[c * FA + k]
  static_assert(2 * NCN <= 2 * NX_ * NY_, "the anti-diagonal fluxes fit the displacements' storage");
};

template <typename R, int NM, int BT, typename T>
__device__ __forceinline__ void dual_tile(const Prob<R> *probs, const BlockMap bm, int gpar) {
  constexpr int TX = T::TX, TY = T::TY;
  using SH = DualShared<R, T>;
  __shared__ SH sh;
  const auto &P = *cst(probs + bm.prob);
  const auto &g = P.g;
  Ctl *ctl = P.ctl;
  const int par = gpar ^ P.flip;
  const Slot &S = ctl->slot[par];
  const int tid = threadIdx.x;
  // read with the tile's first global loads; tested once they are issued
  const bool stop = (ldg(&S.done) | ldg(&ctl->err)) != 0;
  const int nx = g.nx, ny = g.ny;
  const int I0 = bm.i0, J0 = bm.j0;
  const R Dx = R(g.dx), Dy = R(g.dy);

  // The global loads of the owned node (stage 3) and of every staged item
  // (stage 1) are issued before any of them is used, so that the block waits
  // for memory once instead of once per stage and item.
  const int a3 = tid % TX, b3 = tid / TX, I3 = I0 + a3, J3 = J0 + b3;
  const bool own3 = tid < TX * TY && I3 <= nx && J3 <= ny;  // (BT may exceed the tile)
  const int p3 = own3 ? J3 * (nx + 1) + I3 : 0;
  // (loaded from a clamped index on every lane, so that no branch holds
  // them; the owned node's values are used by its own thread only, and its
  // u^{lag} is read from the staged node data)
  R ux3 = ldg(P.ux + p3), uy3 = ldg(P.uy + p3), mp3 = R(0);
  if (!g.kinematic) mp3 = ldg(P.mp + p3);
  // (the corner sound speeds likewise, masked where they are used)
  R cs3[4];
  int cs_ok = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int ci = I3 - 1 + (c & 1), cj = J3 - 1 + (c >> 1);
    const bool ok = own3 && ci >= 0 && cj >= 0 && ci < nx && cj < ny;
    cs3[c] = ldg(P.cs + (ok ? cj * nx + ci : 0));
    cs_ok |= ok ? 1 << c : 0;
  }
  // One loop per kind of staged item, so that a lane without an item of a
  // kind (the tail of each loop, walls) loads nothing for it: the loads sit
  // under branches with no other side, and no other branch writes their
  // registers while they are in flight (with one loop over all kinds the
  // compiler waits for each kind's loads before the next kind's branch).
  // Values of items that have none stay unset; stage 1 writes zero there.
  constexpr int NNODE = SH::NX_ * SH::NY_, NPX = SH::PXW * SH::PXH, NPY = SH::PYW * SH::PYH,
                NPC = SH::PCW * SH::PCH;
  constexpr int ITN = (NNODE + BT - 1) / BT, ITX = (NPX + BT - 1) / BT,
                ITY = (NPY + BT - 1) / BT, ITC = (NPC + BT - 1) / BT;
  R pn[ITN][4], px[ITX], py[ITY], pc[ITC][3];
  if (!g.kinematic) {
#pragma unroll
    for (int it = 0; it < ITN; ++it) {  // node: u^{lag}, u^{n+1/2}
      const int l = tid + it * BT;
      const int I = I0 - 2 + l % SH::NX_, J = J0 - 2 + l / SH::NX_;
      if (l < NNODE && I <= nx + 2 && J <= ny + 2) {
        const int p = refl_node(J, ny) * (nx + 1) + refl_node(I, nx);
        pn[it][0] = ldg(P.uLx + p);
        pn[it][1] = ldg(P.uLy + p);
        pn[it][2] = ldg(P.uhx + p);
        pn[it][3] = ldg(P.uhy + p);
      }
    }
#pragma unroll
    for (int it = 0; it < ITX; ++it) {  // primal x-face mass flux
      const int k = tid + it * BT;
      const int I = I0 - 1 + k % SH::PXW, j = J0 - 1 + k / SH::PXW;
      const int rI = I < 0 ? -I : (I > nx ? 2 * nx - I : I);
      if (k < NPX && I <= nx + 1 && j <= ny && rI != 0 && rI != nx)
        px[it] = ldg(P.MX + (refl_cell(j, ny) * (nx + 1) + rI));
    }
#pragma unroll
    for (int it = 0; it < ITY; ++it) {  // primal y-face mass flux
      const int k = tid + it * BT;
      const int i = I0 - 1 + k % SH::PYW, J = J0 - 1 + k / SH::PYW;
      const int rJ = J < 0 ? -J : (J > ny ? 2 * ny - J : J);
      if (k < NPY && i <= nx && J <= ny + 1 && rJ != 0 && rJ != ny)
        py[it] = ldg(P.MY + (rJ * nx + refl_cell(i, nx)));
    }
#pragma unroll
    for (int it = 0; it < ITC; ++it) {  // corner mass flux and the node's displacement direction
      const int k = tid + it * BT;
      const int I = I0 - 1 + k % SH::PCW, J = J0 - 1 + k / SH::PCW;
      const int rI = refl_node(I, nx), rJ = refl_node(J, ny);
      if (k < NPC && I <= nx + 1 && J <= ny + 1 && rI != 0 && rI != nx && rJ != 0 && rJ != ny) {
        const int p = rJ * (nx + 1) + rI;
        pc[it][0] = ldg(P.MC + p);
        pc[it][1] = ldg(P.uhx + p);
        pc[it][2] = ldg(P.uhy + p);
      }
    }
  }
  bool last;
  const R dt = R(slot_dt(g, S, last));
  if (stop) return;

  if (!g.kinematic) {
    // ---- stage 1: node data and the primal mass fluxes around the tile,
    // mirrored at walls, from the loads issued above
#pragma unroll
    for (int it = 0; it < ITN; ++it) {
      const int l = tid + it * BT;
      const int a = l % SH::NX_, b = l / SH::NX_;
      const int I = I0 - 2 + a, J = J0 - 2 + b;
      if (l >= NNODE || I > nx + 2 || J > ny + 2) continue;
      R ulx = pn[it][0], uly = pn[it][1], dx = dt * pn[it][2], dy = dt * pn[it][3];
      if (refl_node(I, nx) != I) {
        ulx = -ulx;
        dx = -dx;
      }
      if (refl_node(J, ny) != J) {
        uly = -uly;
        dy = -dy;
      }
      sh.ulx[b][a] = ulx;
      sh.uly[b][a] = uly;
      sh.dxy[0][b][a] = dx;
      sh.dxy[1][b][a] = dy;
    }
#pragma unroll
    for (int it = 0; it < ITX; ++it) {
      const int k = tid + it * BT;
      const int a = k % SH::PXW, b = k / SH::PXW;
      const int I = I0 - 1 + a, j = J0 - 1 + b;
      const int rI = I < 0 ? -I : (I > nx ? 2 * nx - I : I);
      if (k >= NPX) continue;
      const bool none = I > nx + 1 || j > ny || rI == 0 || rI == nx;  // wall or outside
      const R sg = (I < 0 || I > nx) ? R(-1) : R(1);  // a mirrored x-face flux changes sign
      sh.mx[b][a] = none ? R(0) : sg * px[it];
    }
#pragma unroll
    for (int it = 0; it < ITY; ++it) {
      const int k = tid + it * BT;
      const int a = k % SH::PYW, b = k / SH::PYW;
      const int i = I0 - 1 + a, J = J0 - 1 + b;
      const int rJ = J < 0 ? -J : (J > ny ? 2 * ny - J : J);
      if (k >= NPY) continue;
      const bool none = i > nx || J > ny + 1 || rJ == 0 || rJ == ny;
      const R sg = (J < 0 || J > ny) ? R(-1) : R(1);
      sh.my[b][a] = none ? R(0) : sg * py[it];
    }
#pragma unroll
    for (int it = 0; it < ITC; ++it) {
      const int k = tid + it * BT;
      const int a = k % SH::PCW, b = k / SH::PCW;
      const int I = I0 - 1 + a, J = J0 - 1 + b;
      if (k >= NPC) continue;
      const bool fx = I < 0 || I > nx, fy = J < 0 || J > ny;
      const int rI = refl_node(I, nx), rJ = refl_node(J, ny);
      const bool none = I > nx + 1 || J > ny + 1 || rI == 0 || rI == nx || rJ == 0 || rJ == ny;
      // (main, anti) pair: the kind from the real node's displacement,
      // then the mirrors (x: (d, a) -> (-a, -d); y: (d, a) -> (a, d))
      const R F = none ? R(0) : pc[it][0];
      R dg = R(0), an = R(0);
      if (corner_main(dt * pc[it][1], dt * pc[it][2])) dg = F;
      else an = F;
      if (fy) { const R t = dg; dg = an; an = t; }
      if (fx) { const R t = dg; dg = -an; an = -t; }
      sh.cd[b][a] = dg;
      sh.ca[b][a] = an;
    }
    __syncthreads();
    auto L = [&](int I) { return I - (I0 - 2); };
    auto M_ = [&](int J) { return J - (J0 - 2); };
    // the dual mesh keeps the limited linear values along each direction
    // with the multidimensional reconstruction of the cell quantities too
    const bool o2 = g.recon_order >= 2;
    // both velocity components at donor node (la, lb), limited slopes along
    // (sa, sb) projected on (vx, vy), offset `off`
    // Lagrangian position of a staged node: its index times the cell size
    // plus its (mirrored) displacement, for ghost nodes too
    auto Xp = [&](int la, int lb) { return R(I0 - 2 + la) * Dx + sh.dxy[0][lb][la]; };
    auto Yp = [&](int la, int lb) { return R(J0 - 2 + lb) * Dy + sh.dxy[1][lb][la]; };
    auto recon = [&](int la, int lb, int sa, int sb, R vx, R vy, R off, R &u, R &v) {
      u = sh.ulx[lb][la];
      v = sh.uly[lb][la];
      if (!o2) return;
      const int ma = la - sa, mb = lb - sb, pa = la + sa, pb = lb + sb;
      const R lm = (Xp(la, lb) - Xp(ma, mb)) * vx + (Yp(la, lb) - Yp(ma, mb)) * vy;
      const R lp = (Xp(pa, pb) - Xp(la, lb)) * vx + (Yp(pa, pb) - Yp(la, lb)) * vy;
      const R su = van_leer_d(u - sh.ulx[mb][ma], sh.ulx[pb][pa] - u, lm, lp);
      const R sv = van_leer_d(v - sh.uly[mb][ma], sh.uly[pb][pa] - v, lm, lp);
      u += su * off;
      v += sv * off;
    };
    auto wxd = [&](int la, int lb) { return Dx + R(0.5) * (sh.dxy[0][lb][la + 1] - sh.dxy[0][lb][la - 1]); };
    auto wyd = [&](int la, int lb) { return Dy + R(0.5) * (sh.dxy[1][lb + 1][la] - sh.dxy[1][lb - 1][la]); };
    const R nrmv = sqrt(Dx * Dx + Dy * Dy);
    const R dgx = Dx / nrmv, dgy = Dy / nrmv;  // unit vector of the main diagonal

    // ---- stage 2: every dual region of the tile once: x-faces, y-faces,
    // then the corners, in one pass.  The anti-diagonal corner fluxes wait in
    // registers until every displacement has been read (a thread meets
    // corners only in its trips from IT2C on), then take the displacements'
    // storage.
    constexpr int NREG = SH::NXF + SH::NYF + SH::NCN, IT2 = (NREG + BT - 1) / BT,
                  IT2C = (SH::NXF + SH::NYF) / BT;
    // regions without mass flux (material at rest) carry no momentum: their
    // fluxes are written as zero without the reconstruction, except in the
    // two-threads-per-node tiles of small FP64 launches, timed by their
    // slowest tile
    constexpr bool REST = BT == T::NT;
    R ha[IT2 - IT2C][2];
    // each region's mass flux, kept for stage 3 (written over the primal
    // fluxes once stage 2 has read them); the anti-diagonal corners' in pa
    R pm[IT2], pa[IT2 - IT2C];
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
      pm[it] = R(0);
      if (it >= IT2C) pa[it - IT2C] = R(0);
    }
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
      const int l = tid + it * BT;
      if (l >= NREG) continue;
      if (l < SH::NXF) {  // dual x-face (I,J): nodes (I-1,J)-(I,J)
        const int a = l % (TX + 1), b = l / (TX + 1);
        const int I = I0 + a, J = J0 + b;
        if (I > nx + 1 || J > ny) continue;
        const R phi = R(0.25) * (sh.mx[b][a] + sh.mx[b][a + 1] + sh.mx[b + 1][a] + sh.mx[b + 1][a + 1]);
        pm[it] = phi;
        if (REST && phi == R(0)) {
          sh.fx[0][l] = R(0);
          sh.fx[1][l] = R(0);
          continue;
        }
        const int D = phi > R(0) ? I - 1 : I;
        const R sg = phi > R(0) ? R(1) : R(-1);
        const R df = R(0.5) * (sh.dxy[0][M_(J)][L(I - 1)] + sh.dxy[0][M_(J)][L(I)]);
        const R off = R(0.5) * (sg * wxd(L(D), M_(J)) - df);
        R u, v;
        recon(L(D), M_(J), 1, 0, R(1), R(0), off, u, v);
        sh.fx[0][l] = phi * u;
        sh.fx[1][l] = phi * v;
      } else if (l < SH::NXF + SH::NYF) {  // dual y-face (I,J): nodes (I,J-1)-(I,J)
        const int k = l - SH::NXF;
        const int a = k % TX, b = k / TX;
        const int I = I0 + a, J = J0 + b;
        if (I > nx || J > ny + 1) continue;
        const R phi = R(0.25) * (sh.my[b][a] + sh.my[b][a + 1] + sh.my[b + 1][a] + sh.my[b + 1][a + 1]);
        pm[it] = phi;
        if (REST && phi == R(0)) {
          sh.fy[0][k] = R(0);
          sh.fy[1][k] = R(0);
          continue;
        }
        const int D = phi > R(0) ? J - 1 : J;
        const R sg = phi > R(0) ? R(1) : R(-1);
        const R df = R(0.5) * (sh.dxy[1][M_(J - 1)][L(I)] + sh.dxy[1][M_(J)][L(I)]);
        const R off = R(0.5) * (sg * wyd(L(I), M_(D)) - df);
        R u, v;
        recon(L(I), M_(D), 0, 1, R(0), R(1), off, u, v);
        sh.fy[0][k] = phi * u;
        sh.fy[1][k] = phi * v;
      } else {  // dual corners at cell (i,j)
        const int k = l - SH::NXF - SH::NYF;
        const int a = k % (TX + 1), b = k / (TX + 1);
        const int i = I0 - 1 + a, j = J0 - 1 + b;
        if (i > nx || j > ny) continue;
        // corner pairs at the cell's nodes (i..i+1, j..j+1): staged at [b..b+1][a..a+1]
        const R d00 = sh.cd[b][a], a00 = sh.ca[b][a], d10 = sh.cd[b][a + 1], a10 = sh.ca[b][a + 1];
        const R d01 = sh.cd[b + 1][a], a01 = sh.ca[b + 1][a], d11 = sh.cd[b + 1][a + 1],
                a11 = sh.ca[b + 1][a + 1];
        const R dcx = R(0.25) * (sh.dxy[0][M_(j)][L(i)] + sh.dxy[0][M_(j)][L(i + 1)] +
                                 sh.dxy[0][M_(j + 1)][L(i)] + sh.dxy[0][M_(j + 1)][L(i + 1)]);
        const R dcy = R(0.25) * (sh.dxy[1][M_(j)][L(i)] + sh.dxy[1][M_(j)][L(i + 1)] +
                                 sh.dxy[1][M_(j + 1)][L(i)] + sh.dxy[1][M_(j + 1)][L(i + 1)]);
        pm[it] = R(0.25) * (d00 + d10 + d01 + d11);
        if (it >= IT2C) pa[it >= IT2C ? it - IT2C : 0] = R(0.25) * (a00 + a10 + a01 + a11);
        if (REST && d00 == R(0) && d10 == R(0) && d01 == R(0) && d11 == R(0)) {
          sh.fd[0][k] = R(0);
          sh.fd[1][k] = R(0);
        } else {  // main diagonal: (i,j) -> (i+1,j+1)
          const R phi = pm[it];
          const R sg = phi > R(0) ? R(1) : R(-1);
          const int DI = phi > R(0) ? i : i + 1, DJ = phi > R(0) ? j : j + 1;
          const R vx = dgx, vy = dgy;
          R u, v, off = R(0);
          if (o2) off = R(0.5) * ((sg * wxd(L(DI), M_(DJ)) - dcx) * vx + (sg * wyd(L(DI), M_(DJ)) - dcy) * vy);
          recon(L(DI), M_(DJ), 1, 1, vx, vy, off, u, v);
          sh.fd[0][k] = phi * u;
          sh.fd[1][k] = phi * v;
        }
        if (REST && a00 == R(0) && a10 == R(0) && a01 == R(0) && a11 == R(0)) {
          if (it >= IT2C) {
            ha[it >= IT2C ? it - IT2C : 0][0] = R(0);
            ha[it >= IT2C ? it - IT2C : 0][1] = R(0);
          }
        } else {  // anti-diagonal: (i,j+1) -> (i+1,j)
          const R phi = pa[it >= IT2C ? it - IT2C : 0];
          const R sg = phi > R(0) ? R(1) : R(-1);
          const int DI = phi > R(0) ? i : i + 1, DJ = phi > R(0) ? j + 1 : j;
          const R vx = dgx, vy = -dgy;
          R u, v, off = R(0);
          if (o2) off = R(0.5) * ((sg * wxd(L(DI), M_(DJ)) - dcx) * vx + (-sg * wyd(L(DI), M_(DJ)) - dcy) * vy);
          recon(L(DI), M_(DJ), 1, -1, vx, vy, off, u, v);
          if (it >= IT2C) {  // (always so for a corner)
            ha[it >= IT2C ? it - IT2C : 0][0] = phi * u;
            ha[it >= IT2C ? it - IT2C : 0][1] = phi * v;
          }
        }
      }
    }
    // the displacements and the primal fluxes are read: the displacements'
    // storage takes the anti-diagonal momentum fluxes, the primal fluxes'
    // the regions' mass fluxes
    __syncthreads();
    R *const fa = &sh.dxy[0][0][0];
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
      const int l = tid + it * BT;
      if (l >= NREG) continue;
      if (l < SH::NXF) {
        (&sh.mx[0][0])[l] = pm[it];
      } else if (l < SH::NXF + SH::NYF) {
        (&sh.my[0][0])[l - SH::NXF] = pm[it];
      } else if (it >= IT2C) {  // (always so for a corner)
        const int k = l - SH::NXF - SH::NYF;
        (&sh.cd[0][0])[k] = pm[it];
        (&sh.ca[0][0])[k] = pa[it - IT2C];
        const int i = I0 - 1 + k % (TX + 1), j = J0 - 1 + k / (TX + 1);
        if (i > nx || j > ny) continue;
        fa[k] = ha[it - IT2C][0];
        fa[SH::FA + k] = ha[it - IT2C][1];
      }
    }
    __syncthreads();
  }

  // ---- stage 3: nodal momentum update, CFL bound of the new state
  unsigned long long cand = ~0ull;
  {
    const int a = a3, b = b3;
    const int I = I3, J = J3;
    if (own3) {
      const int p = p3;
      R ux = ux3, uy = uy3;
      if (!g.kinematic) {
        const int hW = b * (TX + 1) + a, hE = hW + 1;
        const int hS = b * TX + a, hN = hS + TX;
        const int hSW = b * (TX + 1) + a, hNE = (b + 1) * (TX + 1) + a + 1;  // cells (I-1,J-1), (I,J)
        const int hNW = (b + 1) * (TX + 1) + a, hSE = b * (TX + 1) + a + 1;  // cells (I-1,J), (I,J-1)
        // the node's mass and momentum sums, compensated in FP32 as the
        // remap's cell sums are; the node's u^{lag} starts the momentum
        Acc<R> am, au, av;
        am.init(mp3);
        au.init(mp3 * sh.ulx[b + 2][a + 2]);
        av.init(mp3 * sh.uly[b + 2][a + 2]);
        // mass fluxes of the eight dual regions, as stage 2 formed them
        const R *fmx = &sh.mx[0][0], *fmy = &sh.my[0][0], *fmd = &sh.cd[0][0], *fma = &sh.ca[0][0];
        const R *fa = &sh.dxy[0][0][0];  // anti-diagonal fluxes (x at k, y at FA + k)
        am.add(fmx[hW]); au.add(sh.fx[0][hW]); av.add(sh.fx[1][hW]);
        am.add(-fmx[hE]); au.add(-sh.fx[0][hE]); av.add(-sh.fx[1][hE]);
        am.add(fmy[hS]); au.add(sh.fy[0][hS]); av.add(sh.fy[1][hS]);
        am.add(-fmy[hN]); au.add(-sh.fy[0][hN]); av.add(-sh.fy[1][hN]);
        am.add(fmd[hSW]); au.add(sh.fd[0][hSW]); av.add(sh.fd[1][hSW]);
        am.add(-fmd[hNE]); au.add(-sh.fd[0][hNE]); av.add(-sh.fd[1][hNE]);
        am.add(fma[hNW]); au.add(fa[hNW]); av.add(fa[SH::FA + hNW]);
        am.add(-fma[hSE]); au.add(-fa[hSE]); av.add(-fa[SH::FA + hSE]);
        const R m = am.get(), mu = au.get(), mv = av.get();
        if (!(m > R(0))) atomicOr(&ctl->err, ERR_NODEMASS);
        ux = qdiv(mu, m);
        uy = qdiv(mv, m);
        if (I == 0 || I == nx) ux = R(0);
        if (J == 0 || J == ny) uy = R(0);
        if (!isfinite(ux) || !isfinite(uy)) atomicOr(&ctl->err, ERR_NAN);
        stg(P.ux + p, ux);
        stg(P.uy + p, uy);
      }
      // node-wise CFL bound: the largest sound speed of the adjacent cells
      R cmax = R(0);
#pragma unroll
      for (int c = 0; c < 4; ++c) cmax = fmax(cmax, ((cs_ok >> c) & 1) ? cs3[c] : R(0));
      const double bound = fmin(double(Dx / (cmax + fabs(ux))), double(Dy / (cmax + fabs(uy))));
      cand = (unsigned long long)__double_as_longlong(bound);
    }
  }
  block_min_to_slot(cand, ctl->slot[par ^ 1], g.ndt);
}

// one block per tile of the map (LOOP false: grid = map), or a grid smaller
// than the map whose blocks walk it (LOOP true; a separate instantiation,
// since the loop keeps values live across tiles and costs registers)
// WIDE: two threads per node of the tile, so that each thread stages and
// forms half as many items.  For small FP64 launches, where the grid is one
// round of blocks and its time one tile's latency; with many tiles the one-
// thread-per-node form keeps more tiles per CU.
template <typename R, int NM, bool LOOP, bool WIDE, typename T>
__global__ void __launch_bounds__(WIDE ? 2 * T::NT : T::NT)
    k_dual(const Prob<R> *probs, const BlockMap *map, int nmap, int gpar) {
  constexpr int BT = WIDE ? 2 * T::NT : T::NT;
  if constexpr (LOOP) {
    for (int b = blockIdx.x; b < nmap; b += gridDim.x) {
      dual_tile<R, NM, BT, T>(probs, map_entry(map, b), gpar);
      __syncthreads();  // the next tile reuses the LDS
    }
  } else {
    if (blockIdx.x < nmap) dual_tile<R, NM, BT, T>(probs, map_entry(map, xcd_tile(blockIdx.x, nmap)), gpar);
  }
}
// launches of at most this many tiles take the wide FP64 Lagrange and dual
// kernels
constexpr int kWideMaxTiles = 1024;

// ------------------------------------------------------------ kernel table
constexpr int kKernels = 4;
const char *const kKernelNames[kKernels] = {"k_lagrange", "k_mixed", "k_remap", "k_dual"};

template <typename R, int NM, typename T>
struct Resident {  // blocks of each step kernel resident on the whole device
  int n[kKernels] = {0, 0, 0, 0};
  Resident() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return;
    const void *fn[kKernels] = {reinterpret_cast<const void *>(&k_lagrange<R, NM, true, false, T>),
                                reinterpret_cast<const void *>(&k_mixed<R, NM>),
                                reinterpret_cast<const void *>(&k_remap<R, NM, true, true, T>),
                                reinterpret_cast<const void *>(&k_dual<R, NM, true, false, T>)};
    const int bt[kKernels] = {T::NT, NTHREADS, T::NT, T::NT};
    for (int k = 0; k < kKernels; ++k) {
      int per = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn[k], bt[k], 0) == hipSuccess)
        n[k] = per * cus;
    }
  }
};

// blocks per problem of the mixed-cell kernel in a launch of nprob problems
// whose largest has `cells` cells: one 32-cell group per block for up to
// C/512 groups (the list's starting capacity, C/16 cells, in one pass), each
// block striding over the rest.  With many problems the launch is held near
// 2048 blocks: a block with no group still takes a launch slot and reads the
// problem's control record.
inline int mix_chunks_for(long long cells, int nprob = 1) {
  const long long c = cells / 512;
  int n = (int)(c < 16 ? 16 : (c > 1024 ? 1024 : c));
  const int cap = 2048 / (nprob > 0 ? nprob : 1);
  if (n > cap) n = cap < 4 ? 4 : cap;
  return n;
}

template <typename R, int NM, typename T>
const Resident<R, NM, T> &resident() {
  static const Resident<R, NM, T> r;
  return r;
}

// a kernel launch; with ev, a start/stop event pair recorded by the dispatch
// itself (kernel time only, as a kernel trace reports it)
template <typename K, typename... Args>
void launch_b(K kernel, dim3 grid, int block, hipStream_t s, hipEvent_t *ev, Args... args) {
  if (ev) hipExtLaunchKernelGGL(kernel, grid, dim3(block), 0, s, ev[0], ev[1], 0, args...);
  else kernel<<<grid, block, 0, s>>>(args...);
}
template <typename K, typename... Args>
void launch(K kernel, dim3 grid, hipStream_t s, hipEvent_t *ev, Args... args) {
  launch_b(kernel, grid, NTHREADS, s, ev, args...);
}

// one step on tiles of shape T: ev (optional) holds a start/stop pair per
// kernel.  The FP64 forms of small launches with two threads per cell exist
// for the default 32x8 shape and the 32x12 shape of small single grids.
template <typename R, int NM, typename T>
void step_impl(const Launch &L, int gpar, hipStream_t s, hipEvent_t *ev) {
  const Resident<R, NM, T> &res = resident<R, NM, T>();
  const Prob<R> *p = static_cast<const Prob<R> *>(L.probs);
  auto grid = [&](int k, int n) { return (L.persistent && res.n[k] > 0 && res.n[k] < n) ? res.n[k] : n; };
  auto evk = [&](int k) { return ev ? ev + 2 * k : nullptr; };
  const bool loop = L.persistent && res.n[0] > 0 && res.n[1] > 0 && res.n[2] > 0 && res.n[3] > 0;
  const BlockMap *nm = L.node_map, *cm = L.cell_map;
  const int nb = L.node_blocks, cb = L.cell_blocks;
  constexpr bool kWideForm =
      sizeof(R) == 8 && (std::is_same<T, TileDefault>::value || std::is_same<T, TileShape<32, 12>>::value);
  // the Lagrange kernel runs over the cell tiles: node tiles of a boundary
  // node column or row alone would be one thirty-second or one eighth full
  if (loop) {
    launch_b(k_lagrange<R, NM, true, false, T>, dim3(grid(0, cb)), T::NT, s, evk(0), p, cm, cb, gpar);
  } else {
    bool wide = false;
    if constexpr (kWideForm) {
      wide = cb <= kWideMaxTiles;
      if (wide) launch_b(k_lagrange<R, NM, false, true, T>, dim3(cb), 2 * T::NT, s, evk(0), p, cm, cb, gpar);
    }
    if (!wide) launch_b(k_lagrange<R, NM, false, false, T>, dim3(cb), T::NT, s, evk(0), p, cm, cb, gpar);
  }
  launch(k_mixed<R, NM>, dim3(L.mix_chunks, L.nprob), s, evk(1), p, L.plist, gpar);
  if (loop) {
    launch_b(k_remap<R, NM, true, true, T>, dim3(grid(2, cb)), T::NT, s, evk(2), p, cm, cb, gpar);
  } else {
    bool small = false;
    if constexpr (kWideForm) {
      small = cb <= kWideMaxTiles;
      if (small) launch_b(k_remap<R, NM, false, false, T>, dim3(cb), T::NT, s, evk(2), p, cm, cb, gpar);
    }
    if (!small) launch_b(k_remap<R, NM, false, true, T>, dim3(cb), T::NT, s, evk(2), p, cm, cb, gpar);
  }
  if (loop) {
    launch_b(k_dual<R, NM, true, false, T>, dim3(grid(3, nb)), T::NT, s, evk(3), p, nm, nb, gpar);
  } else {
    bool wide = false;
    if constexpr (kWideForm) {
      wide = nb <= kWideMaxTiles;
      if (wide) launch_b(k_dual<R, NM, false, true, T>, dim3(nb), 2 * T::NT, s, evk(3), p, nm, nb, gpar);
    }
    if (!wide) launch_b(k_dual<R, NM, false, false, T>, dim3(nb), T::NT, s, evk(3), p, nm, nb, gpar);
  }
}

// the DirectCF step of a problem of nmat materials on tiles of shape T; the
// resident block counts are queried here, before any stream capture
template <typename R, typename T>
StepFn tiled_step(int nmat) {
  switch (nmat) {
    case 1: (void)resident<R, 1, T>(); return step_impl<R, 1, T>;
    case 2: (void)resident<R, 2, T>(); return step_impl<R, 2, T>;
    case 3: (void)resident<R, 3, T>(); return step_impl<R, 3, T>;
    default: (void)resident<R, 4, T>(); return step_impl<R, 4, T>;
  }
}

}  // namespace
