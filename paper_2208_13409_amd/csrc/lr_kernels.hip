// lr_kernels.hip — the library's main translation unit (gfx950): the
// DirectCF step kernels on the default tile shape, the alternate-direction
// remap, and the host side of the C-ABI declared in include/lr.h (single
// problems, batches, the allocation-free entry point).  The step kernels on
// the other tile shapes are compiled in translation units of their own.
#include "lr_step.hpp"

namespace {

// =========================================================== set-up kernels
template <typename R>
__global__ void k_init_state(Prob<R> P, const double *k, const double *rho, const double *e) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int C = P.g.nx * P.g.ny;
  if (q >= C) return;
  for (int m = 0; m < P.g.nmat; ++m) {
    const int h = m * C + q;
    const double V = k[h] * P.g.A;
    const double M = k[h] > 0.0 ? rho[h] * V : 0.0;
    P.V[0][h] = R(V);
    P.M[0][h] = R(M);
    P.E[0][h] = R(k[h] > 0.0 ? M * e[h] : 0.0);
  }
}
template <typename R>
__global__ void k_init_vel(Prob<R> P, const double *ux, const double *uy) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = (P.g.nx + 1) * (P.g.ny + 1);
  if (p >= N) return;
  const int I = p % (P.g.nx + 1), J = p / (P.g.nx + 1);
  P.ux[p] = (I == 0 || I == P.g.nx) ? R(0) : R(ux[p]);
  P.uy[p] = (J == 0 || J == P.g.ny) ? R(0) : R(uy[p]);
}
// sound speed of the state in buffer `buf`
template <typename R>
__global__ void k_sound(Prob<R> P, int buf) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const Grid &g = P.g;
  const int C = g.nx * g.ny;
  if (q >= C) return;
  R rc2 = R(0), Msum = R(0);
  for (int m = 0; m < g.nmat; ++m) {
    const R V = P.V[buf][m * C + q], M = P.M[buf][m * C + q], E = P.E[buf][m * C + q];
    if (present(g, V)) {
      const R rho = M / V, e = M > R(0) ? E / M : R(0);
      rc2 += eos_krc2(g, m, V / R(g.A), eos_p(g, m, rho, e));
    }
    Msum += M;
  }
  const R rhoc = Msum / R(g.A);
  const R c2 = rhoc > R(0) ? rc2 / rhoc : R(0);
  P.cs[q] = c2 > R(0) ? sqrt(c2) : R(0);
}
// node-wise CFL bound of the current state into slot `slot`
template <typename R>
__global__ void k_dt_bound(Prob<R> P, int slot) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const Grid &g = P.g;
  const int nx = g.nx, ny = g.ny;
  unsigned long long cand = ~0ull;
  if (p < (nx + 1) * (ny + 1)) {
    const int I = p % (nx + 1), J = p / (nx + 1);
    R cmax = R(0);
    for (int bb = -1; bb <= 0; ++bb)
      for (int aa = -1; aa <= 0; ++aa) {
        const int ci = I + aa, cj = J + bb;
        if (ci < 0 || cj < 0 || ci >= nx || cj >= ny) continue;
        cmax = fmax(cmax, P.cs[cj * nx + ci]);
      }
    const double bound = fmin(double(R(g.dx) / (cmax + fabs(P.ux[p]))),
                              double(R(g.dy) / (cmax + fabs(P.uy[p]))));
    cand = (unsigned long long)__double_as_longlong(bound);
  }
  block_min_to_slot(cand, P.ctl->slot[slot], g.ndt);
}

// a device input of element type T copied into the FP64 staging array
template <typename T>
__global__ void k_to_f64(const T *src, double *dst, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = double(src[i]);
}

// the checks of a host-given state, on device arrays k, rho, e [nmat][C]
// and ux, uy [N]; bits: 1 non-finite, 2 fractions outside [0,1] or not
// summing to 1, 4 rho <= 0 or e < 0 where k > 0
__global__ void k_check_state(int nmat, int C, int N, const double *kk, const double *rr,
                              const double *ee, const double *ux, const double *uy, int *bits) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int b = 0;
  if (i < C) {
    double ks = 0.0;
    for (int a = 0; a < nmat; ++a) {
      const double k = kk[(size_t)a * C + i], rho = rr[(size_t)a * C + i], e = ee[(size_t)a * C + i];
      if (!isfinite(k) || !isfinite(rho) || !isfinite(e)) b |= 1;
      if (k < 0.0 || k > 1.0) b |= 2;
      if (k > 0.0 && (!(rho > 0.0) || e < 0.0)) b |= 4;
      ks += k;
    }
    if (!(fabs(ks - 1.0) <= 1e-12)) b |= 2;
  }
  if (i < N && (!isfinite(ux[i]) || !isfinite(uy[i]))) b |= 1;
  if (b) atomicOr(bits, b);
}

// derived output fields of the state in buffer `buf`
template <typename R>
__global__ void k_fields(Prob<R> P, int buf, unsigned bit, double *out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const Grid &g = P.g;
  const int C = g.nx * g.ny, N = (g.nx + 1) * (g.ny + 1);
  if (bit == LR_F_UX || bit == LR_F_UY) {
    if (idx < N) out[idx] = double(bit == LR_F_UX ? P.ux[idx] : P.uy[idx]);
    return;
  }
  if (idx >= C) return;
  const int q = idx;
  double Ms = 0.0, Es = 0.0, Ps = 0.0;
  for (int m = 0; m < g.nmat; ++m) {
    const double V = P.V[buf][m * C + q], M = P.M[buf][m * C + q], E = P.E[buf][m * C + q];
    const bool pr = V > g.k_eps * g.A;
    const double rho = pr ? M / V : 0.0, e = (pr && M > 0.0) ? E / M : 0.0;
    const double Pm = pr ? eos_p(g, m, rho, e) : 0.0;
    Ms += M;
    Es += E;
    Ps += (V / g.A) * Pm;
    double v = 0.0;
    bool per = true;
    switch (bit) {
      case LR_F_K: v = V / g.A; break;
      case LR_F_RHOA: v = rho; break;
      case LR_F_EA: v = e; break;
      case LR_F_PA: v = Pm; break;
      case LR_F_VOL: v = V; break;
      case LR_F_MASS: v = M; break;
      case LR_F_IE: v = E; break;
      default: per = false;
    }
    if (per) out[m * C + q] = v;
  }
  if (bit == LR_F_RHO) out[q] = Ms / g.A;
  if (bit == LR_F_P) out[q] = Ps;
  if (bit == LR_F_E) out[q] = Ms > 0.0 ? Es / Ms : 0.0;
}

// FP64 totals: one partial per block (fixed order), then one thread sums them
template <typename R>
__global__ void k_totals_partial(Prob<R> P, int buf, double *part) {
  const Grid &g = P.g;
  const int nq = 3 * g.nmat + 3;
  const int C = g.nx * g.ny, N = (g.nx + 1) * (g.ny + 1);
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  const int item = blockIdx.x * blockDim.x + tid;
  for (int qq = 0; qq < nq; ++qq) {
    double v = 0.0;
    if (qq < 3 * g.nmat) {
      const int a = qq % g.nmat, kind = qq / g.nmat;
      const R *src = kind == 0 ? P.V[buf] : (kind == 1 ? P.M[buf] : P.E[buf]);
      if (item < C) v = double(src[a * C + item]);
    } else if (item < N) {
      const int I = item % (g.nx + 1), J = item / (g.nx + 1);
      double m = 0.0;
      for (int b = -1; b <= 0; ++b)
        for (int a = -1; a <= 0; ++a) {
          const int ci = I + a, cj = J + b;
          if (ci < 0 || cj < 0 || ci >= g.nx || cj >= g.ny) continue;
          for (int s = 0; s < g.nmat; ++s) m += 0.25 * double(P.M[buf][s * C + cj * g.nx + ci]);
        }
      const double u = double(P.ux[item]), w = double(P.uy[item]);
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
  double et = 0.0;
  for (int a = 0; a < nmat; ++a) et += out[2 * nmat + a];
  out[nq - 1] = et + out[nq - 1];
}

// start a run: the current slot (the larger step) gets t_end and the step
// limit, the other one is stopped until the first step prepares it
__global__ void k_start(Ctl *ctl, double t_end, long long max_steps) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int c = ctl->slot[1].step > ctl->slot[0].step ? 1 : 0;
  Slot &s = ctl->slot[c];
  s.t_end = t_end;
  s.limit = s.step + max_steps;
  s.nmix = 0;
  s.done = (max_steps <= 0 || !(s.t < t_end)) ? 1 : 0;
  ctl->slot[c ^ 1].done = 1;
  ctl->err = 0;
}

}  // namespace

#include "lr_ad.hpp"

namespace {

// the step of a problem: the DirectCF remap, or the alternate-direction one
template <typename R>
StepFn step_fn(int nmat, int remap = LR_REMAP_DIRECTCF) {
  if (remap == LR_REMAP_AD) switch (nmat) {
      case 1: return ad_step_impl<R, 1>;
      case 2: return ad_step_impl<R, 2>;
      case 3: return ad_step_impl<R, 3>;
      default: return ad_step_impl<R, 4>;
    }
  return tiled_step<R, TileDefault>(nmat);
}

// the DirectCF step on tile shape `tile` (LR_TILE_*)
template <typename R>
StepFn step_fn_tile(int nmat, int tile) {
  constexpr int fp32 = sizeof(R) == 4;
  switch (tile) {
    case LR_TILE_16x16: return step_fn_tile16x16(fp32, nmat);
    case LR_TILE_32x16: return step_fn_tile32x16(fp32, nmat);
    case LR_TILE_32x12: return step_fn_tile32x12(fp32, nmat);
    default: return tiled_step<R, TileDefault>(nmat);
  }
}

}  // namespace

#include "lr_host.hpp"
#include "lr_batch.hpp"
#include "lr_noalloc.hpp"
