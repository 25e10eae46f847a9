// lr_host.hpp — host side of the C-ABI declared in include/lr.h (part of the
// lr_kernels.hip translation unit): device allocation of one problem in the
// chosen precision, block maps, device-side time control, outputs.
#pragma once

struct lr_ctx {
  lr_opts o{};
  Grid g{};
  Prob<double> pd{};
  Prob<float> pf{};
  void *dprob = nullptr;  // device copy of the problem descriptor
  BlockMap *node_map = nullptr, *cell_map = nullptr;
  int node_blocks = 0, cell_blocks = 0;
  StepFn step = nullptr;
  Ctl *ctl = nullptr;   // device
  Ctl *hctl = nullptr;  // pinned host mirror
  hipStream_t own = nullptr, stream = nullptr;
  std::vector<void *> allocs;
  bool have_state = false;
  std::string err;
  double *scratch = nullptr;  // staging for outputs
  size_t scratch_n = 0;
  // kernel timing (lr_profile): event marks of the steps of one chunk
  bool prof = false;
  std::vector<hipEvent_t> ev;
  int prof_steps = 0;
  double prof_ms[kKernels] = {0};
  long prof_n[kKernels] = {0};
};

namespace {

constexpr int kChunk = 16;  // steps launched between completion checks

int set_err(lr_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}
#define HIP_CHECK(c, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
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

template <typename R>
int alloc_prob(lr_ctx *c, Prob<R> &P) {
  const Grid &g = c->g;
  const size_t C = (size_t)g.nx * g.ny, N = (size_t)(g.nx + 1) * (g.ny + 1), m = g.nmat;
  const size_t nX = (size_t)(g.nx + 1) * g.ny, nY = (size_t)g.nx * (g.ny + 1);
  P = Prob<R>{};
  P.g = g;
  P.flip = 0;
  int rc = LR_OK;
  for (int b = 0; b < 2; ++b) {
    rc |= dalloc(c, &P.V[b], m * C);
    rc |= dalloc(c, &P.M[b], m * C);
    rc |= dalloc(c, &P.E[b], m * C);
  }
  rc |= dalloc(c, &P.ux, N); rc |= dalloc(c, &P.uy, N);
  rc |= dalloc(c, &P.uhx, N); rc |= dalloc(c, &P.uhy, N);
  rc |= dalloc(c, &P.uLx, N); rc |= dalloc(c, &P.uLy, N); rc |= dalloc(c, &P.mp, N);
  rc |= dalloc(c, &P.eL, m * C);
  rc |= dalloc(c, &P.cs, C);
  rc |= dalloc(c, &P.MX, nX); rc |= dalloc(c, &P.MY, nY); rc |= dalloc(c, &P.MC, N);
  rc |= dalloc(c, &P.mix_cell, C); rc |= dalloc(c, &P.mix_slot, C);
  P.mix_cap = (int)C;
  rc |= dalloc(c, &P.mix_W, C * 8 * m);
  if (c->o.stages) {
    rc |= dalloc(c, &P.dbg.Q, C); rc |= dalloc(c, &P.dbg.S, C); rc |= dalloc(c, &P.dbg.VL, C);
    rc |= dalloc(c, &P.dbg.Ph, m * C); rc |= dalloc(c, &P.dbg.volcf, C);
    rc |= dalloc(c, &P.dbg.rhocf, m * C);
    rc |= dalloc(c, &P.dbg.Wpx, m * nX); rc |= dalloc(c, &P.dbg.Wpy, m * nY);
    rc |= dalloc(c, &P.dbg.Wpc, m * N);
  }
  if (rc != LR_OK) return LR_ENOMEM;
  P.ctl = c->ctl;
  // wall regions are never written: keep them zero
  HIP_CHECK(c, hipMemsetAsync(P.MX, 0, nX * sizeof(R), c->own));
  HIP_CHECK(c, hipMemsetAsync(P.MY, 0, nY * sizeof(R), c->own));
  HIP_CHECK(c, hipMemsetAsync(P.MC, 0, N * sizeof(R), c->own));
  if (P.dbg.Wpx) {
    HIP_CHECK(c, hipMemsetAsync(P.dbg.Wpx, 0, m * nX * sizeof(R), c->own));
    HIP_CHECK(c, hipMemsetAsync(P.dbg.Wpy, 0, m * nY * sizeof(R), c->own));
    HIP_CHECK(c, hipMemsetAsync(P.dbg.Wpc, 0, m * N * sizeof(R), c->own));
  }
  void *d = nullptr;
  if (hipMalloc(&d, sizeof(Prob<R>)) != hipSuccess) return LR_ENOMEM;
  c->allocs.push_back(d);
  c->dprob = d;
  HIP_CHECK(c, hipMemcpyAsync(d, &P, sizeof(Prob<R>), hipMemcpyHostToDevice, c->own));
  c->step = step_fn<R>(g.nmat);
  return LR_OK;
}

int build_maps(lr_ctx *c) {
  const Grid &g = c->g;
  std::vector<BlockMap> nm, cm;
  for (int j = 0; j <= g.ny; j += TY)
    for (int i = 0; i <= g.nx; i += TX) nm.push_back({0, i, j, 0});
  for (int j = 0; j < g.ny; j += TY)
    for (int i = 0; i < g.nx; i += TX) cm.push_back({0, i, j, 0});
  c->node_blocks = (int)nm.size();
  c->cell_blocks = (int)cm.size();
  if (dalloc(c, &c->node_map, nm.size()) || dalloc(c, &c->cell_map, cm.size())) return LR_ENOMEM;
  HIP_CHECK(c, hipMemcpyAsync(c->node_map, nm.data(), nm.size() * sizeof(BlockMap), hipMemcpyHostToDevice, c->own));
  HIP_CHECK(c, hipMemcpyAsync(c->cell_map, cm.data(), cm.size() * sizeof(BlockMap), hipMemcpyHostToDevice, c->own));
  HIP_CHECK(c, hipStreamSynchronize(c->own));
  return LR_OK;
}

bool fp32(const lr_ctx *c) { return c->o.precision == LR_FP32; }

int read_ctl(lr_ctx *c) {
  HIP_CHECK(c, hipMemcpyAsync(c->hctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIP_CHECK(c, hipStreamSynchronize(c->stream));
  return LR_OK;
}
int cur_slot(const Ctl &k) { return k.slot[1].step > k.slot[0].step ? 1 : 0; }

// the time step a slot describes, with the device's arithmetic
double host_slot_dt(const Grid &g, const Slot &s) {
  unsigned long long b = s.dtmin[0];
  for (int k = 1; k < NDT; ++k) b = s.dtmin[k] < b ? s.dtmin[k] : b;
  double dtmin;
  std::memcpy(&dtmin, &b, sizeof dtmin);
  double dt = g.fixed_dt > 0.0 ? g.fixed_dt : g.cfl * dtmin;
  if (s.t_end - s.t <= dt) dt = s.t_end - s.t;
  return dt;
}

int err_code(lr_ctx *c, int bits) {
  if (bits & ERR_NAN) return set_err(c, LR_ENAN, "non-finite value in the state");
  if (bits & ERR_DT) return set_err(c, LR_EDT, "time step not positive or not finite");
  if (bits & ERR_VOLCF) return set_err(c, LR_ENEGATIVE, "flux-consistent Lagrangian volume <= 0");
  if (bits & ERR_NODEMASS) return set_err(c, LR_ENEGATIVE, "nodal mass <= 0 after remap");
  if (bits & ERR_NEG) return set_err(c, LR_ENEGATIVE, "negative partial volume, mass or energy");
  if (bits & ERR_MIXCAP) return set_err(c, LR_ENOMEM, "mixed-cell list capacity exceeded");
  return LR_OK;
}

int collect_profile(lr_ctx *c) {
  if (!c->prof || c->prof_steps == 0) return LR_OK;
  HIP_CHECK(c, hipStreamSynchronize(c->stream));
  for (int st = 0; st < c->prof_steps; ++st)
    for (int k = 0; k < kKernels; ++k) {
      float ms = 0.0f;
      hipEvent_t *e = &c->ev[(size_t)st * (kKernels + 1)];
      HIP_CHECK(c, hipEventElapsedTime(&ms, e[k], e[k + 1]));
      c->prof_ms[k] += ms;
      c->prof_n[k] += 1;
    }
  c->prof_steps = 0;
  return LR_OK;
}

// step until done (t_end reached, max_steps taken, or an error); the host
// checks completion once per chunk of steps
int run_steps(lr_ctx *c, double t_end, long long max_steps) {
  int rc = read_ctl(c);
  if (rc) return rc;
  int gpar = cur_slot(*c->hctl);
  k_start<<<1, 1, 0, c->stream>>>(c->ctl, t_end, max_steps);
  HIP_CHECK(c, hipGetLastError());
  const Launch L{c->dprob, c->node_map, c->cell_map, c->node_blocks, c->cell_blocks};
  for (;;) {
    rc = read_ctl(c);
    if (rc) return rc;
    rc = collect_profile(c);
    if (rc) return rc;
    const Ctl &k = *c->hctl;
    const Slot &s = k.slot[cur_slot(k)];
    if (s.done || k.err) break;
    const long long left = s.limit - s.step;
    const long long n = left < kChunk ? left : kChunk;
    for (long long st = 0; st < n; ++st) {
      hipEvent_t *ev = nullptr;
      if (c->prof && c->prof_steps < kChunk) ev = &c->ev[(size_t)c->prof_steps++ * (kKernels + 1)];
      c->step(L, gpar, c->stream, ev);
      gpar ^= 1;
    }
    HIP_CHECK(c, hipGetLastError());
  }
  return err_code(c, c->hctl->err);
}

template <typename R>
void launch_set_state(lr_ctx *c, Prob<R> &P, const double *dk) {
  const Grid &g = c->g;
  const int C = g.nx * g.ny, N = (g.nx + 1) * (g.ny + 1);
  k_init_state<R><<<(C + 255) / 256, 256, 0, c->stream>>>(P, dk, dk + (size_t)g.nmat * C,
                                                          dk + 2 * (size_t)g.nmat * C);
  k_init_vel<R><<<(N + 255) / 256, 256, 0, c->stream>>>(P, dk + 3 * (size_t)g.nmat * C,
                                                       dk + 3 * (size_t)g.nmat * C + N);
  k_sound<R><<<(C + 255) / 256, 256, 0, c->stream>>>(P, 0);
  k_dt_bound<R><<<(N + 255) / 256, 256, 0, c->stream>>>(P, 0);
}

template <typename R>
int get_fields_impl(lr_ctx *c, Prob<R> &P, int buf, unsigned mask, double *const *out) {
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
    k_fields<R><<<(unsigned)((N + 255) / 256), 256, 0, c->stream>>>(P, buf, bit, c->scratch);
    HIP_CHECK(c, hipGetLastError());
    HIP_CHECK(c, hipMemcpyAsync(o, c->scratch, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  }
  HIP_CHECK(c, hipStreamSynchronize(c->stream));
  return LR_OK;
}

template <typename R>
int totals_impl(lr_ctx *c, Prob<R> &P, int buf, double *out) {
  const Grid &g = c->g;
  const int N = (g.nx + 1) * (g.ny + 1);
  const int nb = (N + 255) / 256, nq = 3 * g.nmat + 3;
  double *part = nullptr;
  HIP_CHECK(c, hipMalloc(&part, ((size_t)nq * nb + nq) * sizeof(double)));
  k_totals_partial<R><<<nb, 256, 0, c->stream>>>(P, buf, part);
  k_totals_final<<<1, 64, 0, c->stream>>>(g.nmat, nb, part, part + (size_t)nq * nb);
  const hipError_t e1 = hipMemcpyAsync(out, part + (size_t)nq * nb, nq * sizeof(double),
                                       hipMemcpyDeviceToHost, c->stream);
  const hipError_t e2 = hipStreamSynchronize(c->stream);
  (void)hipFree(part);
  if (e1 != hipSuccess || e2 != hipSuccess) return set_err(c, LR_EDEVICE, "totals failed");
  return LR_OK;
}

// copy `count` elements of a device array of R into out as doubles
template <typename R>
int copy_out(lr_ctx *c, const R *src, size_t count, double *out) {
  if (!src) return set_err(c, LR_ESTATE, "stage not kept: create the context with opts.stages = 1");
  std::vector<R> h(count);
  HIP_CHECK(c, hipMemcpyAsync(h.data(), src, count * sizeof(R), hipMemcpyDeviceToHost, c->stream));
  HIP_CHECK(c, hipStreamSynchronize(c->stream));
  for (size_t k = 0; k < count; ++k) out[k] = double(h[k]);
  return LR_OK;
}

template <typename R>
int debug_impl(lr_ctx *c, Prob<R> &P, const std::string &n, double *out) {
  const Grid &g = c->g;
  const size_t C = (size_t)g.nx * g.ny, N = (size_t)(g.nx + 1) * (g.ny + 1);
  const size_t nX = (size_t)(g.nx + 1) * g.ny, nY = (size_t)g.nx * (g.ny + 1), m = g.nmat;
  int rc = read_ctl(c);
  if (rc) return rc;
  const Ctl &k = *c->hctl;
  const int cur = cur_slot(k);
  const double dt = host_slot_dt(g, k.slot[cur ^ 1]);
  if (n == "dt") { out[0] = dt; return LR_OK; }
  if (n == "t") { out[0] = k.slot[cur].t; return LR_OK; }
  if (n == "Q") return copy_out(c, P.dbg.Q, C, out);
  if (n == "S") return copy_out(c, P.dbg.S, C, out);
  if (n == "VL") return copy_out(c, P.dbg.VL, C, out);
  if (n == "P_half") return copy_out(c, P.dbg.Ph, m * C, out);
  if (n == "volcf") return copy_out(c, P.dbg.volcf, C, out);
  if (n == "rhocf") return copy_out(c, P.dbg.rhocf, m * C, out);
  if (n == "eL") return copy_out(c, P.eL, m * C, out);
  if (n == "mp") return copy_out(c, P.mp, N, out);
  if (n == "uhx") return copy_out(c, P.uhx, N, out);
  if (n == "uhy") return copy_out(c, P.uhy, N, out);
  if (n == "uLx") return copy_out(c, P.uLx, N, out);
  if (n == "uLy") return copy_out(c, P.uLy, N, out);
  if (n == "muX") return copy_out(c, P.MX, nX, out);
  if (n == "muY") return copy_out(c, P.MY, nY, out);
  if (n == "Wpx") return copy_out(c, P.dbg.Wpx, m * nX, out);
  if (n == "Wpy") return copy_out(c, P.dbg.Wpy, m * nY, out);
  if (n == "Wpc") return copy_out(c, P.dbg.Wpc, m * N, out);
  if (n == "dpx" || n == "dpy" || n == "muD" || n == "muA") {
    std::vector<double> hx(N), hy(N), fc(N);
    rc = copy_out(c, P.uhx, N, hx.data());
    if (!rc) rc = copy_out(c, P.uhy, N, hy.data());
    if (!rc) rc = copy_out(c, P.MC, N, fc.data());
    if (rc) return rc;
    for (size_t p = 0; p < N; ++p) {
      const R dxr = R(dt) * R(hx[p]), dyr = R(dt) * R(hy[p]);
      const bool mainc = (dxr >= R(0)) == (dyr >= R(0));
      if (n == "dpx") out[p] = double(dxr);
      else if (n == "dpy") out[p] = double(dyr);
      else if (n == "muD") out[p] = mainc ? fc[p] : 0.0;
      else out[p] = mainc ? 0.0 : fc[p];
    }
    return LR_OK;
  }
  return set_err(c, LR_EINVAL, "unknown stage name");
}

}  // namespace

extern "C" {

void lr_default_opts(lr_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->x0 = 0; o->x1 = 1; o->y0 = 0; o->y1 = 1;
  o->cfl = 0.5; o->a1 = 0.5; o->a2 = 1.0;
  o->precision = LR_FP64; o->recon_order = 2; o->kinematic = 0;
  o->k_eps = 1e-10; o->fixed_dt = 0.0; o->stages = 0;
}

void lr_destroy(lr_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  for (void *p : c->allocs) (void)hipFree(p);
  if (c->hctl) (void)hipHostFree(c->hctl);
  if (c->own) (void)hipStreamDestroy(c->own);
  delete c;
}

int lr_create(int nx, int ny, int nmat, const lr_eos *eos, const int bc[4], const lr_opts *opts,
              lr_ctx **out) {
  if (!out) return LR_EINVAL;
  *out = nullptr;
  if (nx < 2 || ny < 2 || nmat < 1 || nmat > LR_MAXMAT || !eos) return LR_EINVAL;
  if ((long long)nx * ny > (1ll << 28)) return LR_EINVAL;
  if (bc)
    for (int s = 0; s < 4; ++s)
      if (bc[s] != LR_BC_REFLECT) return LR_EINVAL;
  for (int a = 0; a < nmat; ++a)
    if (!(eos[a].gamma > 1.0) || eos[a].pinf != 0.0) return LR_EINVAL;
  lr_opts o;
  if (opts) o = *opts;
  else lr_default_opts(&o);
  if (!(o.x1 > o.x0) || !(o.y1 > o.y0) || !(o.cfl > 0) || (o.recon_order != 1 && o.recon_order != 2) ||
      !(o.k_eps >= 0) || o.fixed_dt < 0 || (o.precision != LR_FP64 && o.precision != LR_FP32))
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
  // FP32 rounding leaves residues of about 1e-7 of a cell behind a material
  // that moved out: presence and negativity thresholds above that level
  g.neg_tol = o.precision == LR_FP32 ? 1e-5 : 1e-10;
  if (o.precision == LR_FP32 && g.k_eps < 1e-6) g.k_eps = 1e-6;
  for (int a = 0; a < nmat; ++a) g.gamma[a] = eos[a].gamma;
  if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
    lr_destroy(c);
    return LR_EDEVICE;
  }
  c->stream = c->own;
  int rc = dalloc(c, &c->ctl, 1);
  if (rc == LR_OK && hipHostMalloc((void **)&c->hctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess)
    rc = LR_ENOMEM;
  if (rc == LR_OK) rc = fp32(c) ? alloc_prob<float>(c, c->pf) : alloc_prob<double>(c, c->pd);
  if (rc == LR_OK) rc = build_maps(c);
  const size_t N = (size_t)(nx + 1) * (ny + 1), nX = (size_t)(nx + 1) * ny;
  c->scratch_n = std::max((size_t)nmat * std::max(N, nX), (size_t)4096);
  if (rc == LR_OK) rc = dalloc(c, &c->scratch, c->scratch_n);
  if (rc == LR_OK && hipStreamSynchronize(c->own) != hipSuccess) rc = LR_EDEVICE;
  if (rc != LR_OK) {
    lr_destroy(c);
    return rc;
  }
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
  const int nm = g.nmat;
  const size_t C = (size_t)g.nx * g.ny, N = (size_t)(g.nx + 1) * (g.ny + 1);
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
  for (size_t p = 0; p < N; ++p)
    if (!std::isfinite(ux[p]) || !std::isfinite(uy[p])) return set_err(c, LR_ENAN, "non-finite velocity");
  double *dk = nullptr;
  if (hipMalloc(&dk, (3 * nm * C + 2 * N) * sizeof(double)) != hipSuccess)
    return set_err(c, LR_ENOMEM, "staging");
  hipStream_t s = c->stream;
  int rc = LR_OK;
  Ctl h{};
  h.slot[0].t = t;
  h.slot[0].t_end = t;
  const double inf = INFINITY;
  for (int kk = 0; kk < NDT; ++kk) std::memcpy(&h.slot[0].dtmin[kk], &inf, sizeof inf);
  h.slot[0].step = 0;
  h.slot[0].done = 1;
  h.slot[1] = h.slot[0];
  h.slot[1].step = -1;
  *c->hctl = h;
  if (hipMemcpyAsync(dk, k, nm * C * sizeof(double), hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(dk + nm * C, rho, nm * C * sizeof(double), hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(dk + 2 * nm * C, e, nm * C * sizeof(double), hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(dk + 3 * nm * C, ux, N * sizeof(double), hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(dk + 3 * nm * C + N, uy, N * sizeof(double), hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(c->ctl, c->hctl, sizeof(Ctl), hipMemcpyHostToDevice, s)) {
    rc = set_err(c, LR_EDEVICE, "upload failed");
  } else {
    if (fp32(c)) launch_set_state<float>(c, c->pf, dk);
    else launch_set_state<double>(c, c->pd, dk);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      rc = set_err(c, LR_EDEVICE, "initialisation kernels failed");
  }
  (void)hipFree(dk);
  if (rc == LR_OK) c->have_state = true;
  return rc;
}

int lr_step(lr_ctx *c, double *dt_out) {
  if (!c) return LR_EINVAL;
  if (!c->have_state) return set_err(c, LR_ESTATE, "no state set");
  const int rc = run_steps(c, INFINITY, 1);
  if (dt_out) {
    const Ctl &k = *c->hctl;
    *dt_out = host_slot_dt(c->g, k.slot[cur_slot(k) ^ 1]);
  }
  return rc;
}

int lr_run(lr_ctx *c, double t_end, long max_steps, long *steps_out, double *t_out) {
  if (!c) return LR_EINVAL;
  if (!c->have_state) return set_err(c, LR_ESTATE, "no state set");
  int rc = read_ctl(c);
  if (rc) return rc;
  const Ctl &k0 = *c->hctl;
  const Slot s0 = k0.slot[cur_slot(k0)];
  if (!(t_end >= s0.t) || max_steps < 0) return set_err(c, LR_EINVAL, "t_end < t or max_steps < 0");
  rc = run_steps(c, t_end, max_steps);
  const Ctl &k = *c->hctl;
  const Slot &s = k.slot[cur_slot(k)];
  if (steps_out) *steps_out = (long)(s.step - s0.step);
  if (t_out) *t_out = s.t;
  return rc;
}

int lr_get_fields(lr_ctx *c, unsigned mask, double *const *out) {
  if (!c || !out) return LR_EINVAL;
  if (!c->have_state) return set_err(c, LR_ESTATE, "no state set");
  int rc = read_ctl(c);
  if (rc) return rc;
  const int buf = cur_slot(*c->hctl);
  return fp32(c) ? get_fields_impl<float>(c, c->pf, buf, mask, out)
                 : get_fields_impl<double>(c, c->pd, buf, mask, out);
}

int lr_totals(lr_ctx *c, double *out) {
  if (!c || !out) return LR_EINVAL;
  if (!c->have_state) return set_err(c, LR_ESTATE, "no state set");
  int rc = read_ctl(c);
  if (rc) return rc;
  const int buf = cur_slot(*c->hctl);
  return fp32(c) ? totals_impl<float>(c, c->pf, buf, out) : totals_impl<double>(c, c->pd, buf, out);
}

int lr_debug_get(lr_ctx *c, const char *name, double *out) {
  if (!c || !name || !out) return LR_EINVAL;
  if (!c->have_state) return set_err(c, LR_ESTATE, "no state set");
  const std::string n(name);
  return fp32(c) ? debug_impl<float>(c, c->pf, n, out) : debug_impl<double>(c, c->pd, n, out);
}

int lr_profile(lr_ctx *c, int enable) {
  if (!c) return LR_EINVAL;
  if (enable && c->ev.empty()) {
    c->ev.resize((size_t)kChunk * (kKernels + 1));
    for (auto &e : c->ev) HIP_CHECK(c, hipEventCreate(&e));
  }
  c->prof = enable != 0;
  c->prof_steps = 0;
  return LR_OK;
}

int lr_profile_read(lr_ctx *c, double *ms, long *counts, int n) {
  if (!c || n < 0 || n > kKernels) return LR_EINVAL;
  const int rc = collect_profile(c);
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
