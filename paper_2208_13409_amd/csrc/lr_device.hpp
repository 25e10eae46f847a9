// lr_device.hpp — device helpers of the DirectCF Lagrange–Remap kernels
// (gfx950).  Geometry of the flux volumes (paper §2.3), closed-form
// rectangle / half-plane areas and their inverse for the VOF interface (§4.4),
// the Van Leer limited slope (§2.1.1), the wall mirrors, and the per-problem
// descriptors the kernels work on.
#pragma once
#include <hip/hip_runtime.h>

#include "lr.h"

namespace lr {

constexpr int MAXMAT = LR_MAXMAT;
constexpr int NTHREADS = 256;  // block of the kernels that work on lists or whole arrays

// Tile of cells (or nodes) handled by one block of the step kernels, one
// thread per cell.  A single problem takes its shape from its size (32x8,
// 32x12 or 32x16, or the caller's choice); the batch's autotuner times 32x8,
// 16x16 and 32x16 (each shape compiled in a translation unit of its own).
// Every shape computes the same bits: the tile only decides which block
// forms a value, never how.
template <int X, int Y>
struct TileShape {
  static constexpr int TX = X, TY = Y, NT = X * Y;
};
using TileDefault = TileShape<32, 8>;
constexpr int kTileShapes = LR_NTILE;
constexpr int kTileX[kTileShapes] = {32, 16, 32, 32}, kTileY[kTileShapes] = {8, 16, 16, 12};

// Problem constants (FP64 whatever the bulk precision).
struct Grid {
  int nx, ny, nmat;
  int recon_order, kinematic;
  double dx, dy, A;  // cell sizes and area
  double Lx, Ly;     // domain extents x1-x0, y1-y0
  double x0, x1, y0, y1;  // domain
  double cfl, a1, a2, k_eps, fixed_dt;
  double neg_tol;  // a partial V, M, E below -neg_tol of the cell scale is an error
  double gamma[MAXMAT];
  double pinf[MAXMAT];  // stiffened-gas pi (0: perfect gas)
  int ndt;  // CFL partial minima the problem uses (a power of two, 32..NDT)
  int remap;  // LR_REMAP_DIRECTCF or LR_REMAP_AD
  int mix_list;  // requested initial capacity of the mixed-cell list (0: automatic)
};

// Device-side time control.  Step n of a problem reads slot[n & 1 ^ flip];
// the remap kernel of step n prepares the other slot for step n+1 and the
// dual kernel of step n accumulates the CFL bound of the new state into it,
// so no control kernel and no host round trip is needed between steps.
// A launch folds each block's CFL bound into one of the problem's g.ndt
// partial minima (block b into b % g.ndt): device-wide atomics on one address
// are served one after another, so a large grid needs many partials (about
// 16 blocks each), while a small one reads fewer in every kernel's prologue.
constexpr int NDT = 256;
static_assert(NDT % 64 == 0, "each lane of a wave reads NDT / 64 partials");
// partials for a grid of nx x ny cells: 32, doubled while there are more
// than 16 node tiles per partial, at most NDT
inline int cfl_partials(int nx, int ny) {
  const long long tiles = (long long)((nx + TileDefault::TX) / TileDefault::TX) *
                          ((ny + TileDefault::TY) / TileDefault::TY);
  int n = 32;
  while (n < NDT && 16ll * n < tiles) n *= 2;
  return n;
}
struct Slot {
  double t;                       // time at the start of the step
  double t_end;                   // end of the current run
  unsigned long long dtmin[NDT];  // bits of the CFL bound of the state at t (positive
                                  // doubles): its min over the entries; those at or
                                  // beyond the problem's count stay +inf
  long long step;                 // index of the step
  long long limit;                // the run stops when step reaches it
  int done;                       // no step to take: the kernels return at once
  int nmix;                       // mixed cells listed for this step
};
struct Ctl {
  Slot slot[2];
  int err;  // sticky error bits (ERR_*), cleared when a run starts
  int pad;
};
enum { ERR_NEG = 1, ERR_NAN = 2, ERR_DT = 4, ERR_VOLCF = 8, ERR_NODEMASS = 16, ERR_MIXCAP = 32 };

// Optional stage arrays, written only when non-null (stage-by-stage checks).
template <typename R>
struct Dbg {
  R *Q, *S, *VL, *Ph;       // [C], [C], [C], [nmat][C]
  R *volcf, *rhocf;         // [C], [nmat][C]
  R *dxL, *dyL;             // [C] widths of the Lagrangian cell's rectangle
  R *Wpx, *Wpy, *Wpc;       // per-material signed partial volumes of the regions
};

// Arrays of the alternate-direction remap (allocated for it only): the
// state and nodal velocity between its two passes, and each pass's per-cell
// and per-face intermediates (faces of the pass's direction).
template <typename R>
struct AdArrays {
  R *V, *M, *E;          // [nmat][C] state after the first pass
  R *ux, *uy;            // [N] nodal velocity after the first pass
  R *k, *e, *rhocf;      // [nmat][C] pass input fractions, specific energies, rho^{lag}
  R *vol, *cen, *wid;    // [C] pass Lagrangian volume, centre and width along the direction
  R *Mc;                 // [C] mixture mass of the pass input
  int *pure;             // [C] the single present material, or -1
  R *W, *mu, *eps;       // [nmat][faces] partial volume, mass and energy flux of each face
  R *muF;                // [faces] signed total mass flux of each face
};

// Everything a kernel needs to step one problem (device pointers).
template <typename R>
struct Prob {
  Grid g;
  int flip;                       // slot parity of step 0
  R *V[2], *M[2], *E[2];          // [nmat][C] conserved partial volume, mass, internal energy,
                                  // double-buffered by slot: step in slot p reads [p], writes [p^1]
  R *ux, *uy;                     // [N] nodal velocity
  R *uhx, *uhy, *uLx, *uLy, *mp;  // [N] u^{n+1/2}, u^{lag}, nodal mass
  R *eL;                          // [nmat][C] specific internal energy at the end of Lagrange
  R *cs;                          // [C] sound speed of the updated state
  R *MX, *MY, *MC;                // signed total mass flux of x-faces, y-faces, corners
  int *mix_cell, *mix_slot;       // compacted mixed cells; cell -> list position or -1
  int mix_cap;                    // capacity of mix_cell and mix_W (grows on overflow)
  R *mix_W;                       // [mix_cap][8][nmat] outflow partial volumes (formed in
                                  // FP64, stored in the bulk precision)
  Ctl *ctl;
  Dbg<R> dbg;
  AdArrays<R> ad;
};

// block -> (problem, tile origin) of one launch over a batch
struct BlockMap {
  int prob, i0, j0, n;  // n: blocks of this problem (list kernels)
};

// one step's launches: the block maps of node and cell tiles of every
// problem; `persistent` limits each grid to the blocks the device holds at
// once (each block then walks the map)
struct Launch {
  const void *probs;
  const BlockMap *node_map, *cell_map;
  int node_blocks, cell_blocks;
  const int *plist;  // the problems of the launch (for the mixed-cell kernel)
  int nprob;
  int mix_chunks;    // blocks per problem of the mixed-cell kernel
  bool persistent;
  long long cells, nodes;  // of the problem (single-problem launches of the AD remap)
};
using StepFn = void (*)(const Launch &, int, hipStream_t, hipEvent_t *);
// the DirectCF step on the tile shapes other than the default, for a bulk
// precision (fp32: 1) and a material count; each defined in its own
// translation unit
StepFn step_fn_tile16x16(int fp32, int nmat);
StepFn step_fn_tile32x16(int fp32, int nmat);
StepFn step_fn_tile32x12(int fp32, int nmat);
// Workgroups are dispatched to the eight XCDs in turn (block b to XCD b % 8),
// each XCD with its own L2.  Block b takes map entry xcd_tile(b, n) instead of
// b, so that each XCD works through a contiguous run of the map and
// neighbouring tiles, which read each other's halos, share an L2.  A
// bijection of [0, n): XCD x gets entries [x q + min(x, r), ...) with
// q = n / 8, r = n % 8, the first r XCDs one more.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
  return x * q + (x < r ? x : r) + k;
}
// entry b of a block map, read through the constant address space
__device__ __forceinline__ BlockMap map_entry(const BlockMap *map, int b) {
  const auto &m = *(const __attribute__((address_space(4))) BlockMap *)(map + b);
  return BlockMap{m.prob, m.i0, m.j0, m.n};
}

// ---------------------------------------------------------------- memory
// Loads and stores through the arrays of a problem descriptor.  The pointers
// are read from device memory, so the compiler cannot tell global memory from
// LDS and would issue flat instructions, whose completion counter is shared
// with LDS operations; the cast makes them global-memory instructions.
template <typename T>
__device__ __forceinline__ T ldg(const T *p) {
  return *(const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ void stg(T *p, T v) {
  *(__attribute__((address_space(1))) T *)p = v;
}
// Problem descriptors and block maps do not change during a launch: read
// through the constant address space they become scalar loads, kept in
// scalar registers instead of being re-read by every lane after each barrier.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *cst(const T *p) {
  return (const __attribute__((address_space(4))) T *)p;
}

// ---------------------------------------------------------------- arithmetic
// Quotient in the bulk precision: IEEE division in FP64; in FP32 the
// hardware reciprocal (1 ulp) times the numerator, within 2 ulp of the
// rounded quotient, instead of the ten-instruction correctly rounded
// sequence.  The FP64 islands keep IEEE division, and so do quotients by a
// value that may be a float denormal (the reciprocal would overflow).
template <typename R>
__device__ __forceinline__ R qdiv(R a, R b) {
  return a / b;
}
template <>
__device__ __forceinline__ float qdiv<float>(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
}

// ---------------------------------------------------------------- indexing
__device__ __forceinline__ int refl_cell(int i, int n) {
  return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i);
}
__device__ __forceinline__ int refl_node(int I, int n) {
  return I < 0 ? -I : (I > n ? 2 * n - I : I);
}

// ---------------------------------------------------------------- limiter
// Van Leer (the limiter of §2.1.1): for one-sided slopes dm, dp of the same
// sign the harmonic mean 2 dm dp / (dm + dp), otherwise 0.  Taken here from the
// differences to the neighbours, dm_ = a - a_minus and dp_ = a_plus - a, and
// the distances lm, lp to them (dm = dm_/lm, dp = dp_/lp):
// 2 dm dp / (dm + dp) = 2 dm_ dp_ / (dm_ lp + dp_ lm), one quotient instead of three.
template <typename R>
__device__ __forceinline__ R van_leer_d(R dm_, R dp_, R lm, R lp) {
  return (dm_ * dp_) * (lm * lp) > R(0) ? qdiv(R(2) * dm_ * dp_, dm_ * lp + dp_ * lm) : R(0);
}

// ---------------------------------------------------------------- geometry
// Quadrilateral area F of §1.2 from node positions relative to a common origin:
// half the absolute cross product of the left and bottom edges plus half that
// of the right and top edges.
template <typename R>
__device__ __forceinline__ R quad_area(R blx, R bly, R brx, R bry, R tlx, R tly, R trx, R try_) {
  const R lx = tlx - blx, ly = tly - bly;
  const R bx = brx - blx, by = bry - bly;
  const R rx = trx - brx, ry = try_ - bry;
  const R tx = trx - tlx, ty = try_ - tly;
  return R(0.5) * fabs(lx * by - ly * bx) + R(0.5) * fabs(rx * ty - ry * tx);
}

// F - A as the exact polynomial in the node displacements of a non-inverted
// cell of sides (Dx, Dy): free of the cancellation of F - A in FP32.
template <typename R>
__device__ __forceinline__ R quad_area_change(R Dx, R Dy, R blx, R bly, R brx, R bry, R tlx, R tly,
                                              R trx, R try_) {
  // triangle BL-BR-TL: (Dx + brx - blx)(Dy + tly - bly) - (bry - bly)(tlx - blx) - Dx Dy
  const R b1x = brx - blx, l1y = tly - bly, b1y = bry - bly, l1x = tlx - blx;
  const R t1 = Dx * l1y + Dy * b1x + b1x * l1y - b1y * l1x;
  // triangle TR-TL-BR: (Dy + try - bry)(Dx + trx - tlx) - (trx - brx)(try - tly) - Dx Dy
  const R r2y = try_ - bry, t2x = trx - tlx, r2x = trx - brx, t2y = try_ - tly;
  const R t2 = Dx * r2y + Dy * t2x + r2y * t2x - r2x * t2y;
  return R(0.5) * (t1 + t2);
}

// DirectCF face flux volume (§2.3) of a face of length D whose end nodes are
// displaced by (da_n, da_t) at the lower end and (db_n, db_t) at the upper end
// (n: component normal to the face, t: along it).  The trapezoid between the
// Eulerian face and the Lagrangian face line, cut at t- = max(0, da_t) and
// t+ = D + min(0, db_t), is replaced by a rectangle of width w (the mean
// offset of the line at t-, t+) and height h; the flux volume is w h.
template <typename R>
struct FaceGeo {
  R w;   // signed width: > 0 flux along +n
  R h;   // height (>= 0)
  R t0;  // start of the rectangle along the face, from the lower node
};
template <typename R>
__device__ __forceinline__ FaceGeo<R> face_geo(R da_n, R da_t, R db_n, R db_t, R D) {
  const R tlo = fmax(R(0), da_t);
  const R thi = D + fmin(R(0), db_t);
  R h = thi - tlo;
  if (h < R(0)) h = R(0);
  const R slope = qdiv(db_n - da_n, (D + db_t) - da_t);
  const R nlo = da_n + (tlo - da_t) * slope;
  const R nhi = da_n + (thi - da_t) * slope;
  FaceGeo<R> g;
  g.w = R(0.5) * (nlo + nhi);
  g.h = h;
  g.t0 = tlo;
  return g;
}

// The eight flux regions touching a cell: W, E, S, N faces, then the corners
// at its BL, BR, TL, TR nodes (§2.3, donor table of §3.3).  role: +1 the cell
// is the donor, -1 the receiver, 0 not involved (corner of the other diagonal).
template <typename R>
struct CellRegions {
  FaceGeo<R> fg[4];
  R vol[8];
  int role[8];
};
template <typename R>
__device__ __forceinline__ void cell_regions(R Dx, R Dy, R blx, R bly, R brx, R bry, R tlx, R tly,
                                             R trx, R try_, CellRegions<R> &r) {
  r.fg[0] = face_geo(blx, bly, tlx, tly, Dy);  // W face: normal x, lower node BL
  r.fg[1] = face_geo(brx, bry, trx, try_, Dy);  // E face
  r.fg[2] = face_geo(bly, blx, bry, brx, Dx);  // S face: normal y, left node BL
  r.fg[3] = face_geo(tly, tlx, try_, trx, Dx);  // N face
#pragma unroll
  for (int s = 0; s < 4; ++s) r.vol[s] = fabs(r.fg[s].w * r.fg[s].h);
  r.role[0] = r.fg[0].w >= R(0) ? -1 : 1;
  r.role[1] = r.fg[1].w >= R(0) ? 1 : -1;
  r.role[2] = r.fg[2].w >= R(0) ? -1 : 1;
  r.role[3] = r.fg[3].w >= R(0) ? 1 : -1;
  const R cx[4] = {blx, brx, tlx, trx}, cy[4] = {bly, bry, tly, try_};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    r.vol[4 + s] = fabs(cx[s] * cy[s]);
    const bool sx = cx[s] >= R(0), sy = cy[s] >= R(0);
    int role;
    if (s == 0) role = (sx == sy) ? (sx ? -1 : 1) : 0;       // cell is NE of its BL node
    else if (s == 1) role = (sx != sy) ? (sx ? 1 : -1) : 0;  // NW of its BR node
    else if (s == 2) role = (sx != sy) ? (sx ? -1 : 1) : 0;  // SE of its TL node
    else role = (sx == sy) ? (sx ? 1 : -1) : 0;              // SW of its TR node
    r.role[4 + s] = role;
  }
}
// corner kind at a node: main diagonal when both displacement signs agree
template <typename R>
__device__ __forceinline__ bool corner_main(R dx, R dy) {
  return (dx >= R(0)) == (dy >= R(0));
}

// Area of the part of the rectangle [x0,x1] x [y0,y1] where nx x + ny y >= s,
// in closed form.  With the rectangle centred (half sizes a, b), P = |nx|,
// Q = |ny| and t = P a + Q b - |s'| (depth of the cut below the far corner),
// the cut-off piece is a triangle t^2/(2PQ) while the line meets two adjacent
// sides, and a trapezoid 2a(t - aP)/Q or 2b(t - bQ)/P once it meets two
// opposite sides; s' < 0 uses the complement.  Written without branches, the
// case picking the numerator and denominator of the one quotient: a lane that
// forms several of these areas (one per material) then overlaps their
// latencies instead of running them one after another.
__device__ __forceinline__ double rect_halfplane_area(double x0, double x1, double y0, double y1,
                                                      double nx, double ny, double s) {
  const double a = 0.5 * (x1 - x0), b = 0.5 * (y1 - y0);
  const double sc = s - (nx * (0.5 * (x0 + x1)) + ny * (0.5 * (y0 + y1)));
  const double P = fabs(nx), Q = fabs(ny);
  const double h = P * a + Q * b;
  const double full = 4.0 * a * b;
  const double whole = (x1 - x0) * (y1 - y0);
  const double t = sc >= 0.0 ? h - sc : h + sc;
  const bool xfirst = a * P <= b * Q;  // the line leaves the x-range first
  const bool tri = t <= (xfirst ? 2.0 * a * P : 2.0 * b * Q);
  const double num = tri ? t * t : (xfirst ? 2.0 * a * (t - a * P) : 2.0 * b * (t - b * Q));
  const double den = tri ? 2.0 * P * Q : (xfirst ? Q : P);
  const double piece = t <= 0.0 ? 0.0 : num / den;
  double area = sc >= 0.0 ? piece : full - piece;
  area = area < 0.0 ? 0.0 : (area > whole ? whole : area);
  area = sc >= h ? 0.0 : (sc <= -h ? whole : area);
  return (x1 > x0 && y1 > y0) ? area : 0.0;
}

// Inverse of the cut-off piece's area for T in [0, 2ab]: the depth t giving
// area T (the triangle's root while T stays below the area Tt at which the
// triangle spans the first range the line leaves, the trapezoid's beyond).
// The three candidate quotients and the root are formed side by side and one
// is selected: no branch waits on the quotient Tt.
__device__ __forceinline__ double corner_depth(double a, double b, double P, double Q, double T) {
  const bool xfirst = a * P <= b * Q;
  const double Tt = xfirst ? 2.0 * a * a * P / Q : 2.0 * b * b * Q / P;
  const double root = sqrt(2.0 * P * Q * T);
  const double trap = xfirst ? T * Q / (2.0 * a) + a * P : T * P / (2.0 * b) + b * Q;
  return T <= 0.0 ? 0.0 : (T <= Tt ? root : trap);
}

// Offset s of the line n.x = s such that the part of the rectangle where
// n.x >= s has area frac*|R| (§4.4, placement of the interface), in closed
// form from the piecewise-quadratic area; frac in [0,1], n a unit vector.
// Past half the rectangle the complement's depth is taken, and negated.
__device__ __forceinline__ double interface_offset(double x0, double x1, double y0, double y1,
                                                   double nx, double ny, double frac) {
  const double a = 0.5 * (x1 - x0), b = 0.5 * (y1 - y0);
  const double P = fabs(nx), Q = fabs(ny);
  const double h = P * a + Q * b;
  const double full = 4.0 * a * b;
  const double T = frac * full;
  const bool lower = T <= 0.5 * full;
  const double d = h - corner_depth(a, b, P, Q, lower ? T : full - T);
  const double sc = lower ? d : -d;
  return sc + (nx * (0.5 * (x0 + x1)) + ny * (0.5 * (y0 + y1)));
}

// time step of the step a slot describes (the CFL bound or the fixed step,
// shortened to land on t_end)
// the block's minimum of a per-thread bound (bits of a positive double) goes
// to one of the nd partial minima of the slot: one atomic per block
__device__ __forceinline__ void block_min_to_slot(unsigned long long cand, Slot &s, int nd) {
  __shared__ unsigned long long wmin[16];
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(cand, o, 64);
    cand = w < cand ? w : cand;
  }
  const int wave = threadIdx.x / 64, nw = (blockDim.x + 63) / 64;
  if (__lane_id() == 0) wmin[wave] = cand;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = wmin[0];
    for (int k = 1; k < nw; ++k) m = wmin[k] < m ? wmin[k] : m;
    if (m != ~0ull) atomicMin(&s.dtmin[blockIdx.x & (nd - 1)], m);
  }
}

// (called by all 64 lanes of every wave: lane l reads partial l & 31 at once,
// waiting for no other load; with more than 32 partials also l, l + 64, ...
// below the count, and one more exchange step joins the two halves of the
// wave before the five that give every lane the minimum)
template <typename GridT>
__device__ __forceinline__ double slot_dt(const GridT &g, const Slot &s, bool &last) {
  unsigned long long b = ldg(&s.dtmin[__lane_id() & 31]);
  if (g.ndt > 32) {  // (a multiple of 64)
#pragma unroll
    for (int k = 0; k < NDT / 64; ++k) {
      if (64 * k >= g.ndt) break;
      const unsigned long long v = ldg(&s.dtmin[64 * k + __lane_id()]);
      b = v < b ? v : b;
    }
    const unsigned long long w = __shfl_xor(b, 32, 64);
    b = w < b ? w : b;
  }
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(b, o, 64);
    b = w < b ? w : b;
  }
  const double dtmin = __longlong_as_double((long long)b);
  const double t = ldg(&s.t), t_end = ldg(&s.t_end);
  double dt = g.fixed_dt > 0.0 ? g.fixed_dt : g.cfl * dtmin;
  last = false;
  if (t_end - t <= dt) {
    dt = t_end - t;
    last = true;
  }
  return dt;
}

}  // namespace lr
