// lr_host.hpp — host side of the single-problem C-ABI declared in
// include/lr.h (part of the lr_kernels.hip translation unit), and the helpers
// it shares with the batch: layout of one problem's device arrays, grid and
// state checks, block maps, device-side time control, outputs.
#pragma once

namespace {

constexpr int kChunk = 16;  // steps launched between completion checks

#define HIP_TRY(err, call)                                                      \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      (err) = std::string(#call ": ") + hipGetErrorString(e_);                  \
      return LR_EDEVICE;                                                        \
    }                                                                           \
  } while (0)

// ------------------------------------------------------------ problem layout
// All device arrays of one problem in one allocation, each 256-byte aligned.
// With base == nullptr only the size is computed.
struct Carver {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += (n ? n : 1) * sizeof(T);
    return p;
  }
};

template <typename R>
size_t carve_prob(Prob<R> &P, char *base, const Grid &g, bool stages, Ctl *ctl) {
  const size_t C = (size_t)g.nx * g.ny, N = (size_t)(g.nx + 1) * (g.ny + 1), m = g.nmat;
  const size_t nX = (size_t)(g.nx + 1) * g.ny, nY = (size_t)g.nx * (g.ny + 1);
  Carver cv{base};
  P = Prob<R>{};
  P.g = g;
  P.flip = 0;
  for (int b = 0; b < 2; ++b) {
    P.V[b] = cv.take<R>(m * C);
    P.M[b] = cv.take<R>(m * C);
    P.E[b] = cv.take<R>(m * C);
  }
  P.ux = cv.take<R>(N); P.uy = cv.take<R>(N);
  P.uhx = cv.take<R>(N); P.uhy = cv.take<R>(N);
  P.uLx = cv.take<R>(N); P.uLy = cv.take<R>(N); P.mp = cv.take<R>(N);
  P.eL = cv.take<R>(m * C);
  P.cs = cv.take<R>(C);
  P.MX = cv.take<R>(nX); P.MY = cv.take<R>(nY); P.MC = cv.take<R>(N);
  P.mix_slot = cv.take<int>(C);  // the list itself (mix_cell, mix_W) is carved by carve_list
  if (g.remap == LR_REMAP_AD) {
    const size_t nF = std::max(nX, nY);
    AdArrays<R> &a = P.ad;
    a.V = cv.take<R>(m * C); a.M = cv.take<R>(m * C); a.E = cv.take<R>(m * C);
    a.ux = cv.take<R>(N); a.uy = cv.take<R>(N);
    a.k = cv.take<R>(m * C); a.e = cv.take<R>(m * C); a.rhocf = cv.take<R>(m * C);
    a.vol = cv.take<R>(C); a.cen = cv.take<R>(C); a.wid = cv.take<R>(C); a.Mc = cv.take<R>(C);
    a.pure = cv.take<int>(C);
    a.W = cv.take<R>(m * nF); a.mu = cv.take<R>(m * nF); a.eps = cv.take<R>(m * nF);
    a.muF = cv.take<R>(nF);
  }
  if (stages) {
    P.dbg.Q = cv.take<R>(C); P.dbg.S = cv.take<R>(C); P.dbg.VL = cv.take<R>(C);
    P.dbg.Ph = cv.take<R>(m * C); P.dbg.volcf = cv.take<R>(C);
    P.dbg.rhocf = cv.take<R>(m * C);
    P.dbg.dxL = cv.take<R>(C); P.dbg.dyL = cv.take<R>(C);
    P.dbg.Wpx = cv.take<R>(m * nX); P.dbg.Wpy = cv.take<R>(m * nY);
    P.dbg.Wpc = cv.take<R>(m * N);
  }
  P.ctl = ctl;
  return (cv.off + 255) & ~size_t(255);
}

// The list of mixed cells and their outflow partial volumes, sized to need:
// a separate allocation (or pool range) that grows when a step finds more
// mixed cells than it holds.
inline long long count_mixed_host(const Grid &g, const double *k) {
  const size_t C = (size_t)g.nx * g.ny;
  long long n = 0;
  for (size_t q = 0; q < C; ++q) {
    int np = 0;
    for (int a = 0; a < g.nmat; ++a) np += k[a * C + q] > g.k_eps;
    n += np >= 2;
  }
  return n;
}
// initial capacity: as asked, else the larger of C/16, 256 and twice the
// mixed cells of the initial state (at most C)
inline int mix_cap_initial(const Grid &g, long long nmix0) {
  const long long C = (long long)g.nx * g.ny;
  const long long cap = g.mix_list > 0 ? g.mix_list : std::max(std::max(C / 16, 256ll), 2 * nmix0);
  return (int)std::min(cap, C);
}
// capacity after a step needed `need` entries
inline int mix_cap_grown(const Grid &g, int cap, long long need) {
  const long long C = (long long)g.nx * g.ny;
  return (int)std::min(C, std::max(2ll * cap, need + need / 4 + 64));
}
template <typename R>
size_t carve_list(Prob<R> &P, char *base, const Grid &g, int cap) {
  Carver cv{base};
  P.mix_cell = cv.take<int>((size_t)cap);
  P.mix_W = cv.take<R>((size_t)cap * 8 * g.nmat);
  P.mix_cap = cap;
  return (cv.off + 255) & ~size_t(255);
}
template <typename R>
size_t list_bytes(const Grid &g, int cap) {
  Prob<R> P{};
  return carve_list(P, nullptr, g, cap);
}

// wall regions are never written: keep them zero (outside any graph)
template <typename R>
int clear_prob(const Prob<R> &P, hipStream_t s, std::string &err) {
  const Grid &g = P.g;
  const size_t N = (size_t)(g.nx + 1) * (g.ny + 1), m = g.nmat;
  const size_t nX = (size_t)(g.nx + 1) * g.ny, nY = (size_t)g.nx * (g.ny + 1);
  HIP_TRY(err, hipMemsetAsync(P.MX, 0, nX * sizeof(R), s));
  HIP_TRY(err, hipMemsetAsync(P.MY, 0, nY * sizeof(R), s));
  HIP_TRY(err, hipMemsetAsync(P.MC, 0, N * sizeof(R), s));
  if (P.dbg.Wpx) {
    HIP_TRY(err, hipMemsetAsync(P.dbg.Wpx, 0, m * nX * sizeof(R), s));
    HIP_TRY(err, hipMemsetAsync(P.dbg.Wpy, 0, m * nY * sizeof(R), s));
    HIP_TRY(err, hipMemsetAsync(P.dbg.Wpc, 0, m * N * sizeof(R), s));
  }
  return LR_OK;
}

// ------------------------------------------------------------ checks
int make_grid(int nx, int ny, int nmat, const lr_eos *eos, const int bc[4], const lr_opts &o,
              Grid &g) {
  if (nx < 2 || ny < 2 || nmat < 1 || nmat > LR_MAXMAT || !eos) return LR_EINVAL;
  if ((long long)nx * ny > (1ll << 28)) return LR_EINVAL;
  if (bc)
    for (int s = 0; s < 4; ++s)
      if (bc[s] != LR_BC_REFLECT) return LR_EINVAL;
  for (int a = 0; a < nmat; ++a)
    if (!(eos[a].gamma > 1.0) || !(eos[a].pinf >= 0.0) || !std::isfinite(eos[a].pinf)) return LR_EINVAL;
  if (!(o.x1 > o.x0) || !(o.y1 > o.y0) || !(o.cfl > 0) || o.recon_order < 1 || o.recon_order > 3 ||
      (o.remap == LR_REMAP_AD && o.recon_order == 3) ||
      !(o.k_eps >= 0) || o.fixed_dt < 0 || (o.precision != LR_FP64 && o.precision != LR_FP32) ||
      (o.remap != LR_REMAP_DIRECTCF && o.remap != LR_REMAP_AD) || o.mix_list < 0)
    return LR_EINVAL;
  g = Grid{};
  g.nx = nx; g.ny = ny; g.nmat = nmat;
  g.recon_order = o.recon_order; g.kinematic = o.kinematic ? 1 : 0;
  g.dx = (o.x1 - o.x0) / nx; g.dy = (o.y1 - o.y0) / ny; g.A = g.dx * g.dy;
  g.Lx = o.x1 - o.x0; g.Ly = o.y1 - o.y0;
  g.x0 = o.x0; g.x1 = o.x1; g.y0 = o.y0; g.y1 = o.y1;
  g.remap = o.remap;
  g.mix_list = o.mix_list;
  g.cfl = o.cfl; g.a1 = o.a1; g.a2 = o.a2; g.k_eps = o.k_eps; g.fixed_dt = o.fixed_dt;
  // FP32 rounding leaves residues of about 1e-7 of a cell behind a material
  // that moved out: presence and negativity thresholds above that level
  g.neg_tol = o.precision == LR_FP32 ? 1e-5 : 1e-10;
  if (o.precision == LR_FP32 && g.k_eps < 1e-6) g.k_eps = 1e-6;
  for (int a = 0; a < nmat; ++a) {
    g.gamma[a] = eos[a].gamma;
    g.pinf[a] = eos[a].pinf;
  }
  g.ndt = cfl_partials(nx, ny);
  return LR_OK;
}

// the host checks of an initial state; LR_OK or the code, with *msg
int check_state_host(const Grid &g, const double *k, const double *rho, const double *e,
                     const double *ux, const double *uy, const char **msg) {
  const int nm = g.nmat;
  const size_t C = (size_t)g.nx * g.ny, N = (size_t)(g.nx + 1) * (g.ny + 1);
  for (size_t q = 0; q < C; ++q) {
    double ks = 0.0;
    for (int a = 0; a < nm; ++a) {
      const size_t h = a * C + q;
      if (!std::isfinite(k[h]) || !std::isfinite(rho[h]) || !std::isfinite(e[h])) {
        *msg = "non-finite input";
        return LR_ENAN;
      }
      if (k[h] < 0.0 || k[h] > 1.0) {
        *msg = "volume fraction outside [0,1]";
        return LR_ESTATE;
      }
      if (k[h] > 0.0 && (!(rho[h] > 0.0) || e[h] < 0.0)) {
        *msg = "rho <= 0 or e < 0 where k > 0";
        return LR_ESTATE;
      }
      ks += k[h];
    }
    if (std::fabs(ks - 1.0) > 1e-12) {
      *msg = "volume fractions do not sum to 1";
      return LR_ESTATE;
    }
  }
  for (size_t p = 0; p < N; ++p)
    if (!std::isfinite(ux[p]) || !std::isfinite(uy[p])) {
      *msg = "non-finite velocity";
      return LR_ENAN;
    }
  return LR_OK;
}

// control record of a fresh state at time t: slot 0 is current and runs
// until t_end or `limit` steps; slot 1 is stopped until the first step
Ctl initial_ctl(double t, double t_end, long long limit) {
  Ctl h{};
  h.slot[0].t = t;
  h.slot[0].t_end = t_end;
  const double inf = INFINITY;
  for (int kk = 0; kk < NDT; ++kk) std::memcpy(&h.slot[0].dtmin[kk], &inf, sizeof inf);
  h.slot[0].step = 0;
  h.slot[0].limit = limit;
  h.slot[0].done = (limit <= 0 || !(t < t_end)) ? 1 : 0;
  h.slot[1] = h.slot[0];
  h.slot[1].step = -1;
  h.slot[1].done = 1;
  return h;
}

int cur_slot(const Ctl &k) { return k.slot[1].step > k.slot[0].step ? 1 : 0; }

// the time step a slot describes, with the device's arithmetic
double host_slot_dt(const Grid &g, const Slot &s) {
  unsigned long long b = s.dtmin[0];
  for (int k = 1; k < g.ndt; ++k) b = s.dtmin[k] < b ? s.dtmin[k] : b;
  double dtmin;
  std::memcpy(&dtmin, &b, sizeof dtmin);
  double dt = g.fixed_dt > 0.0 ? g.fixed_dt : g.cfl * dtmin;
  if (s.t_end - s.t <= dt) dt = s.t_end - s.t;
  return dt;
}

int err_code(int bits, const char **msg) {
  if (bits & ERR_NAN) { *msg = "non-finite value in the state"; return LR_ENAN; }
  if (bits & ERR_DT) { *msg = "time step not positive or not finite"; return LR_EDT; }
  if (bits & ERR_VOLCF) { *msg = "flux-consistent Lagrangian volume <= 0"; return LR_ENEGATIVE; }
  if (bits & ERR_NODEMASS) { *msg = "nodal mass <= 0 after remap"; return LR_ENEGATIVE; }
  if (bits & ERR_NEG) { *msg = "negative partial volume, mass or energy"; return LR_ENEGATIVE; }
  if (bits & ERR_MIXCAP) { *msg = "mixed-cell list capacity exceeded"; return LR_ENOMEM; }
  return LR_OK;
}

// node tiles cover nodes [0, nx] x [0, ny], cell tiles cells [0, nx) x [0, ny);
// tiles of tx x ty
void tile_maps(const Grid &g, int prob, std::vector<BlockMap> &nm, std::vector<BlockMap> &cm,
               int tx = TileDefault::TX, int ty = TileDefault::TY) {
  for (int j = 0; j <= g.ny; j += ty)
    for (int i = 0; i <= g.nx; i += tx) nm.push_back({prob, i, j, 0});
  for (int j = 0; j < g.ny; j += ty)
    for (int i = 0; i < g.nx; i += tx) cm.push_back({prob, i, j, 0});
}

// initial state from the FP64 staging array [k | rho | e | ux | uy]:
// conserved totals in buffer 0, sound speed, CFL bound into slot 0
template <typename R>
void launch_init(const Prob<R> &P, const double *dk, hipStream_t s) {
  const Grid &g = P.g;
  const size_t C = (size_t)g.nx * g.ny, N = (size_t)(g.nx + 1) * (g.ny + 1);
  const unsigned cb = (unsigned)((C + 255) / 256), nb = (unsigned)((N + 255) / 256);
  k_init_state<R><<<cb, 256, 0, s>>>(P, dk, dk + g.nmat * C, dk + 2 * g.nmat * C);
  k_init_vel<R><<<nb, 256, 0, s>>>(P, dk + 3 * g.nmat * C, dk + 3 * g.nmat * C + N);
  k_sound<R><<<cb, 256, 0, s>>>(P, 0);
  k_dt_bound<R><<<nb, 256, 0, s>>>(P, 0);
}

// doubles of field `bit` of a grid
inline size_t field_count(const Grid &g, unsigned bit) {
  const size_t C = (size_t)g.nx * g.ny, N = (size_t)(g.nx + 1) * (g.ny + 1);
  const bool node = bit == LR_F_UX || bit == LR_F_UY;
  const bool per = bit == LR_F_K || bit == LR_F_RHOA || bit == LR_F_EA || bit == LR_F_PA ||
                   bit == LR_F_VOL || bit == LR_F_MASS || bit == LR_F_IE;
  return node ? N : (per ? g.nmat * C : C);
}

// fields of the state in buffer `buf` into host arrays, through `stage`
// (device, at least max(nmat*C, N) doubles) and, when given, `hstage`
// (pinned host memory for all the fields asked for: the copies then run
// asynchronously on `s` alone, and the host copies out after them)
template <typename R>
int fields_out(const Prob<R> &P, int buf, unsigned mask, double *const *out, double *stage,
               double *hstage, hipStream_t s, std::string &err) {
  const Grid &g = P.g;
  const size_t N = (size_t)(g.nx + 1) * (g.ny + 1);
  int slot = 0;
  size_t off = 0;
  for (unsigned bit = 1; bit <= LR_F_IE; bit <<= 1) {
    if (!(mask & bit)) continue;
    double *o = out[slot++];
    if (!o) {
      err = "null output pointer";
      return LR_EINVAL;
    }
    const size_t n = field_count(g, bit);
    k_fields<R><<<(unsigned)((N + 255) / 256), 256, 0, s>>>(P, buf, bit, stage);
    HIP_TRY(err, hipGetLastError());
    HIP_TRY(err, hipMemcpyAsync(hstage ? hstage + off : o, stage, n * sizeof(double), hipMemcpyDeviceToHost, s));
    off += n;
  }
  HIP_TRY(err, hipStreamSynchronize(s));
  if (hstage) {
    slot = 0;
    off = 0;
    for (unsigned bit = 1; bit <= LR_F_IE; bit <<= 1) {
      if (!(mask & bit)) continue;
      const size_t n = field_count(g, bit);
      std::memcpy(out[slot++], hstage + off, n * sizeof(double));
      off += n;
    }
  }
  return LR_OK;
}

template <typename R>
int totals_out(const Prob<R> &P, int buf, double *out, hipStream_t s, std::string &err) {
  const Grid &g = P.g;
  const int N = (g.nx + 1) * (g.ny + 1);
  const int nb = (N + 255) / 256, nq = 3 * g.nmat + 3;
  double *part = nullptr;
  HIP_TRY(err, hipMalloc(&part, ((size_t)nq * nb + nq) * sizeof(double)));
  k_totals_partial<R><<<nb, 256, 0, s>>>(P, buf, part);
  k_totals_final<<<1, 64, 0, s>>>(g.nmat, nb, part, part + (size_t)nq * nb);
  const hipError_t e1 = hipMemcpyAsync(out, part + (size_t)nq * nb, nq * sizeof(double),
                                       hipMemcpyDeviceToHost, s);
  const hipError_t e2 = hipStreamSynchronize(s);
  (void)hipFree(part);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    err = "totals failed";
    return LR_EDEVICE;
  }
  return LR_OK;
}

}  // namespace

// ============================================================ single problem
struct lr_ctx {
  lr_opts o{};
  Grid g{};
  Prob<double> pd{};
  Prob<float> pf{};
  void *dprob = nullptr;  // device copy of the problem descriptor
  BlockMap *node_map = nullptr, *cell_map = nullptr;
  int node_blocks = 0, cell_blocks = 0;
  int *plist = nullptr;  // device {0}: the problem list of the mixed-cell launch
  StepFn step = nullptr;
  int tile = LR_TILE_32x8;  // tile shape of the step kernels (LR_TILE_*)
  Ctl *ctl = nullptr;   // device
  Ctl *hctl = nullptr;  // pinned host mirror [3]: the context's, then two for
                        // the chunks of a run in flight
  hipEvent_t ctl_ev[2] = {nullptr, nullptr};  // ... their copies done
  hipGraphExec_t chunk_graph[2] = {nullptr, nullptr};  // a full chunk from parity 0 / 1
  bool graph_failed = false;  // capture refused: chunks are launched directly
  char *list_mem = nullptr;   // the mixed-cell list (its own allocation: it grows)
  hipStream_t own = nullptr, stream = nullptr;
  std::vector<void *> allocs;
  bool have_state = false;
  std::string err;
  double *outbuf = nullptr;  // staging for outputs
  // kernel timing (lr_profile): a start/stop event pair per kernel of each
  // step of one chunk
  bool prof = false;
  std::vector<hipEvent_t> ev;
  int prof_steps = 0;
  double prof_ms[kKernels] = {0};
  long prof_n[kKernels] = {0};
};

namespace {

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

template <typename T>
int dalloc(lr_ctx *c, T **p, size_t n) {
  void *q = nullptr;
  if (hipMalloc(&q, (n ? n : 1) * sizeof(T)) != hipSuccess) return LR_ENOMEM;
  c->allocs.push_back(q);
  *p = static_cast<T *>(q);
  return LR_OK;
}

bool fp32(const lr_ctx *c) { return c->o.precision == LR_FP32; }

// the context's mixed-cell list with room for `cap` cells (the old one
// freed: nothing may be queued that reads it), and the device descriptor
template <typename R>
int ctx_list(lr_ctx *c, Prob<R> &P, int cap) {
  HIP_CHECK(c, hipStreamSynchronize(c->stream));
  if (c->list_mem) (void)hipFree(c->list_mem);
  c->list_mem = nullptr;
  if (hipMalloc((void **)&c->list_mem, list_bytes<R>(c->g, cap)) != hipSuccess)
    return set_err(c, LR_ENOMEM, "mixed-cell list");
  carve_list(P, c->list_mem, c->g, cap);
  HIP_CHECK(c, hipMemcpyAsync(c->dprob, &P, sizeof(Prob<R>), hipMemcpyHostToDevice, c->stream));
  HIP_CHECK(c, hipStreamSynchronize(c->stream));
  return LR_OK;
}
int ctx_list_grow(lr_ctx *c, int cap) {
  return fp32(c) ? ctx_list<float>(c, c->pf, cap) : ctx_list<double>(c, c->pd, cap);
}
int ctx_list_cap(const lr_ctx *c) { return fp32(c) ? c->pf.mix_cap : c->pd.mix_cap; }

template <typename R>
int alloc_prob(lr_ctx *c, Prob<R> &P) {
  const size_t bytes = carve_prob(P, nullptr, c->g, c->o.stages != 0, c->ctl);
  char *mem = nullptr;
  if (dalloc(c, &mem, bytes)) return LR_ENOMEM;
  carve_prob(P, mem, c->g, c->o.stages != 0, c->ctl);
  const int rc = clear_prob(P, c->own, c->err);
  if (rc) return rc;
  Prob<R> *d = nullptr;
  if (dalloc(c, &d, 1)) return LR_ENOMEM;
  c->dprob = d;
  HIP_CHECK(c, hipStreamSynchronize(c->own));
  c->step = c->g.remap == LR_REMAP_AD ? step_fn<R>(c->g.nmat, c->g.remap) : step_fn_tile<R>(c->g.nmat, c->tile);
  return ctx_list<R>(c, P, mix_cap_initial(c->g, 0));
}

// LR_TILE_AUTO, by the grid's node tiles against the device's CUs: a grid
// whose 32x8 tiles take one round of blocks keeps them; one whose 32x12 tiles
// do (and 32x8 would not) steps on 32x12, one block per CU (on 32x8 some CUs
// would hold two blocks of the one latency-bound round and set every kernel's
// time); larger grids step on 32x16 (less halo per owned cell, several rounds).
int auto_tile(const Grid &g) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return LR_TILE_32x8;
  auto node_tiles = [&](int t) {
    return (long long)(g.nx / kTileX[t] + 1) * (long long)(g.ny / kTileY[t] + 1);
  };
  if (node_tiles(LR_TILE_32x8) <= cus) return LR_TILE_32x8;
  return node_tiles(LR_TILE_32x12) <= cus ? LR_TILE_32x12 : LR_TILE_32x16;
}

int build_maps(lr_ctx *c) {
  std::vector<BlockMap> nm, cm;
  tile_maps(c->g, 0, nm, cm, kTileX[c->tile], kTileY[c->tile]);
  c->node_blocks = (int)nm.size();
  c->cell_blocks = (int)cm.size();
  if (dalloc(c, &c->node_map, nm.size()) || dalloc(c, &c->cell_map, cm.size()) || dalloc(c, &c->plist, 1))
    return LR_ENOMEM;
  HIP_CHECK(c, hipMemsetAsync(c->plist, 0, sizeof(int), c->own));
  HIP_CHECK(c, hipMemcpyAsync(c->node_map, nm.data(), nm.size() * sizeof(BlockMap), hipMemcpyHostToDevice, c->own));
  HIP_CHECK(c, hipMemcpyAsync(c->cell_map, cm.data(), cm.size() * sizeof(BlockMap), hipMemcpyHostToDevice, c->own));
  HIP_CHECK(c, hipStreamSynchronize(c->own));
  return LR_OK;
}

int read_ctl(lr_ctx *c) {
  HIP_CHECK(c, hipMemcpyAsync(c->hctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIP_CHECK(c, hipStreamSynchronize(c->stream));
  return LR_OK;
}

int ctx_err(lr_ctx *c, int bits) {
  const char *msg = "";
  const int rc = err_code(bits, &msg);
  return rc ? set_err(c, rc, msg) : LR_OK;
}

int collect_profile(lr_ctx *c) {
  if (!c->prof || c->prof_steps == 0) return LR_OK;
  HIP_CHECK(c, hipStreamSynchronize(c->stream));
  for (int st = 0; st < c->prof_steps; ++st)
    for (int k = 0; k < kKernels; ++k) {
      float ms = 0.0f;
      hipEvent_t *e = &c->ev[(size_t)st * 2 * kKernels];
      HIP_CHECK(c, hipEventElapsedTime(&ms, e[2 * k], e[2 * k + 1]));
      c->prof_ms[k] += ms;
      c->prof_n[k] += 1;
    }
  c->prof_steps = 0;
  return LR_OK;
}

Launch ctx_launch(const lr_ctx *c) {
  return Launch{c->dprob,  c->node_map, c->cell_map, c->node_blocks, c->cell_blocks, c->plist, 1,
                mix_chunks_for((long long)c->g.nx * c->g.ny), false, (long long)c->g.nx * c->g.ny,
                (long long)(c->g.nx + 1) * (c->g.ny + 1)};
}

// a full chunk of kChunk steps from parity gpar, replayed from a HIP graph
// captured at its first use (launched directly if the capture fails)
int launch_chunk_graph(lr_ctx *c, int gpar) {
  hipGraphExec_t &x = c->chunk_graph[gpar];
  if (!x) {
    const Launch L = ctx_launch(c);
    hipGraph_t graph = nullptr;
    HIP_CHECK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    for (int st = 0; st < kChunk; ++st) c->step(L, gpar ^ (st & 1), c->stream, nullptr);
    const hipError_t le = hipGetLastError();
    const hipError_t e = hipStreamEndCapture(c->stream, &graph);
    if (le != hipSuccess || e != hipSuccess || !graph ||
        hipGraphInstantiate(&x, graph, nullptr, nullptr, 0) != hipSuccess) {
      x = nullptr;
      c->graph_failed = true;
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (!x) {  // the same steps, launched directly
      for (int st = 0; st < kChunk; ++st) c->step(L, gpar ^ (st & 1), c->stream, nullptr);
      HIP_CHECK(c, hipGetLastError());
      return LR_OK;
    }
  }
  HIP_CHECK(c, hipGraphLaunch(x, c->stream));
  return LR_OK;
}

// step until done (t_end reached, max_steps taken, or an error).  Chunks of
// kChunk steps; chunk k+1 is queued before the host reads chunk k's control
// record (copied after it into one of two pinned mirrors), so the device
// does not wait for the host between chunks.  A chunk queued after the run
// ended (at t_end, which the host learns only from the record) does nothing:
// its kernels see the done flag and return.  Full chunks replay a HIP graph,
// except while kernels are timed.
//
// A step that finds more mixed cells than the list holds sets ERR_MIXCAP in
// its Lagrange kernel; the step's other kernels and every later one then
// return at once, so the state and the step's control slot are those of the
// step's start, except the slot's mixed-cell count and done flag (the later
// steps, returning, mark both slots done).  The list grows to the count the
// step found, the record is restored and the run goes on from that step.
int run_steps(lr_ctx *c, double t_end, long long max_steps) {
  int rc = read_ctl(c);
  if (rc) return rc;
  int gpar = cur_slot(*c->hctl);
  {
    const Slot &s0 = c->hctl->slot[gpar];
    if (max_steps <= 0 || c->hctl->err || s0.t >= t_end) {
      k_start<<<1, 1, 0, c->stream>>>(c->ctl, t_end, max_steps);
      HIP_CHECK(c, hipGetLastError());
      rc = read_ctl(c);
      return rc ? rc : ctx_err(c, c->hctl->err);
    }
  }
  k_start<<<1, 1, 0, c->stream>>>(c->ctl, t_end, max_steps);
  HIP_CHECK(c, hipGetLastError());
  const Launch L = ctx_launch(c);
  for (hipEvent_t &e : c->ctl_ev)
    if (!e) HIP_CHECK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  long long left = max_steps;  // steps still to launch
  for (;;) {
    long long queued = 0;  // steps launched in this pass (at most left)
    int chunk = 0, pending = 0;
    for (;;) {
      if (queued < left) {
        const long long rest = left - queued;
        const int n = rest < kChunk ? (int)rest : kChunk;
        if (n == kChunk && !c->prof && !c->graph_failed) {
          rc = launch_chunk_graph(c, gpar);
          if (rc) return rc;
        } else {
          for (int st = 0; st < n; ++st) {
            hipEvent_t *ev = nullptr;
            if (c->prof && c->prof_steps < kChunk) ev = &c->ev[(size_t)c->prof_steps++ * 2 * kKernels];
            c->step(L, gpar ^ (st & 1), c->stream, ev);
          }
          HIP_CHECK(c, hipGetLastError());
        }
        gpar ^= n & 1;
        queued += n;
        const int m = chunk & 1;
        HIP_CHECK(c, hipMemcpyAsync(c->hctl + 1 + m, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
        HIP_CHECK(c, hipEventRecord(c->ctl_ev[m], c->stream));
        ++chunk;
        ++pending;
        if (c->prof) {  // timed chunks one at a time: the event pairs are reused
          rc = collect_profile(c);
          if (rc) return rc;
        }
        if (pending < 2 && queued < left) continue;  // keep two chunks in flight
      }
      // the oldest chunk in flight: its record says whether the run goes on
      const int m = (chunk - pending) & 1;
      HIP_CHECK(c, hipEventSynchronize(c->ctl_ev[m]));
      --pending;
      const Ctl &k = c->hctl[1 + m];
      if (k.slot[cur_slot(k)].done || k.err || (queued >= left && pending == 0)) break;
    }
    rc = read_ctl(c);  // the record after everything queued
    if (rc) return rc;
    rc = collect_profile(c);
    if (rc) return rc;
    Ctl &k = *c->hctl;
    if (k.err != ERR_MIXCAP) break;
    const int par = cur_slot(k);
    rc = ctx_list_grow(c, mix_cap_grown(c->g, ctx_list_cap(c), k.slot[par].nmix));
    if (rc) return rc;
    k.err = 0;
    k.slot[par].nmix = 0;
    k.slot[par].done = 0;
    HIP_CHECK(c, hipMemcpyAsync(c->ctl, c->hctl, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
    gpar = par;
    left = k.slot[par].limit - k.slot[par].step;
  }
  return ctx_err(c, c->hctl->err);
}

// the state staged as FP64 [k | rho | e | ux | uy] in device memory becomes
// the problem's state at time t
int ctx_init_from_stage(lr_ctx *c, double t, const double *dk) {
  *c->hctl = initial_ctl(t, t, 0);
  HIP_CHECK(c, hipMemcpyAsync(c->ctl, c->hctl, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
  if (fp32(c)) launch_init<float>(c->pf, dk, c->stream);
  else launch_init<double>(c->pd, dk, c->stream);
  HIP_CHECK(c, hipGetLastError());
  HIP_CHECK(c, hipStreamSynchronize(c->stream));
  c->have_state = true;
  return LR_OK;
}

template <typename R>
int debug_copy(lr_ctx *c, const R *src, size_t count, double *out) {
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
  if (n == "run") {
    out[0] = P.mix_cap;
    out[1] = c->chunk_graph[0] || c->chunk_graph[1] ? 1.0 : 0.0;
    out[2] = c->graph_failed ? 1.0 : 0.0;
    out[3] = c->tile;
    return LR_OK;
  }
  if (n == "t") { out[0] = k.slot[cur].t; return LR_OK; }
  if (n == "Q") return debug_copy(c, P.dbg.Q, C, out);
  if (n == "S") return debug_copy(c, P.dbg.S, C, out);
  if (n == "VL") return debug_copy(c, P.dbg.VL, C, out);
  if (n == "P_half") return debug_copy(c, P.dbg.Ph, m * C, out);
  if (n == "volcf") return debug_copy(c, P.dbg.volcf, C, out);
  if (n == "rhocf") return debug_copy(c, P.dbg.rhocf, m * C, out);
  if (n == "dxL") return debug_copy(c, P.dbg.dxL, C, out);
  if (n == "dyL") return debug_copy(c, P.dbg.dyL, C, out);
  if (n == "eL") return debug_copy(c, P.eL, m * C, out);
  if (n == "mp") return debug_copy(c, P.mp, N, out);
  if (n == "uhx") return debug_copy(c, P.uhx, N, out);
  if (n == "uhy") return debug_copy(c, P.uhy, N, out);
  if (n == "uLx") return debug_copy(c, P.uLx, N, out);
  if (n == "uLy") return debug_copy(c, P.uLy, N, out);
  if (n == "muX") return debug_copy(c, P.MX, nX, out);
  if (n == "muY") return debug_copy(c, P.MY, nY, out);
  if (n == "Wpx") return debug_copy(c, P.dbg.Wpx, m * nX, out);
  if (n == "Wpy") return debug_copy(c, P.dbg.Wpy, m * nY, out);
  if (n == "Wpc") return debug_copy(c, P.dbg.Wpc, m * N, out);
  if (n == "dpx" || n == "dpy" || n == "muD" || n == "muA") {
    std::vector<double> hx(N), hy(N), fc(N);
    rc = debug_copy(c, P.uhx, N, hx.data());
    if (!rc) rc = debug_copy(c, P.uhy, N, hy.data());
    if (!rc) rc = debug_copy(c, P.MC, N, fc.data());
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
  o->k_eps = 1e-10; o->fixed_dt = 0.0; o->stages = 0; o->remap = LR_REMAP_DIRECTCF;
  o->tile = LR_TILE_AUTO;
}

void lr_destroy(lr_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ctl_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipGraphExec_t x : c->chunk_graph)
    if (x) (void)hipGraphExecDestroy(x);
  if (c->list_mem) (void)hipFree(c->list_mem);
  for (void *p : c->allocs) (void)hipFree(p);
  if (c->hctl) (void)hipHostFree(c->hctl);
  if (c->own) (void)hipStreamDestroy(c->own);
  delete c;
}

int lr_create(int nx, int ny, int nmat, const lr_eos *eos, const int bc[4], const lr_opts *opts,
              lr_ctx **out) {
  if (!out) return LR_EINVAL;
  *out = nullptr;
  lr_opts o;
  if (opts) o = *opts;
  else lr_default_opts(&o);
  Grid g;
  if (make_grid(nx, ny, nmat, eos, bc, o, g) != LR_OK) return LR_EINVAL;
  if (o.tile < LR_TILE_AUTO || o.tile >= LR_NTILE || (o.remap == LR_REMAP_AD && o.tile > LR_TILE_32x8))
    return LR_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return LR_EDEVICE;
  lr_ctx *c = new (std::nothrow) lr_ctx();
  if (!c) return LR_ENOMEM;
  c->o = o;
  c->g = g;
  c->tile = o.tile != LR_TILE_AUTO ? o.tile : (o.remap == LR_REMAP_AD ? LR_TILE_32x8 : auto_tile(g));
  if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
    lr_destroy(c);
    return LR_EDEVICE;
  }
  c->stream = c->own;
  int rc = dalloc(c, &c->ctl, 1);
  if (rc == LR_OK && hipHostMalloc((void **)&c->hctl, 3 * sizeof(Ctl), hipHostMallocDefault) != hipSuccess)
    rc = LR_ENOMEM;
  if (rc == LR_OK) rc = fp32(c) ? alloc_prob<float>(c, c->pf) : alloc_prob<double>(c, c->pd);
  if (rc == LR_OK) rc = build_maps(c);
  const size_t N = (size_t)(nx + 1) * (ny + 1), C = (size_t)nx * ny;
  if (rc == LR_OK) rc = dalloc(c, &c->outbuf, std::max((size_t)nmat * C, N));
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
  const char *msg = "";
  const int chk = check_state_host(g, k, rho, e, ux, uy, &msg);
  if (chk) return set_err(c, chk, msg);
  const int cap = mix_cap_initial(g, count_mixed_host(g, k));
  if (cap > ctx_list_cap(c)) {
    const int rl = ctx_list_grow(c, cap);
    if (rl) return rl;
  }
  double *dk = nullptr;
  if (hipMalloc(&dk, (3 * nm * C + 2 * N) * sizeof(double)) != hipSuccess)
    return set_err(c, LR_ENOMEM, "staging");
  hipStream_t s = c->stream;
  int rc = LR_OK;
  if (hipMemcpyAsync(dk, k, nm * C * sizeof(double), hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(dk + nm * C, rho, nm * C * sizeof(double), hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(dk + 2 * nm * C, e, nm * C * sizeof(double), hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(dk + 3 * nm * C, ux, N * sizeof(double), hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(dk + 3 * nm * C + N, uy, N * sizeof(double), hipMemcpyHostToDevice, s))
    rc = set_err(c, LR_EDEVICE, "upload failed");
  else
    rc = ctx_init_from_stage(c, t, dk);
  (void)hipStreamSynchronize(s);
  (void)hipFree(dk);
  return rc;
}

int lr_set_state_device(lr_ctx *c, double t, const void *k, const void *rho, const void *e,
                        const void *ux, const void *uy, int dtype) {
  if (!c || !k || !rho || !e || !ux || !uy || (dtype != LR_F64 && dtype != LR_F32)) return LR_EINVAL;
  if (!std::isfinite(t)) return set_err(c, LR_EINVAL, "t not finite");
  const Grid &g = c->g;
  const int nm = g.nmat;
  const size_t C = (size_t)g.nx * g.ny, N = (size_t)(g.nx + 1) * (g.ny + 1);
  const size_t nd = 3 * nm * C + 2 * N;
  double *dk = nullptr;
  if (hipMalloc(&dk, nd * sizeof(double) + 256) != hipSuccess) return set_err(c, LR_ENOMEM, "staging");
  int *bits = reinterpret_cast<int *>(dk + nd);
  hipStream_t s = c->stream;
  const void *src[5] = {k, rho, e, ux, uy};
  const size_t cnt[5] = {nm * C, nm * C, nm * C, N, N};
  size_t off = 0;
  int rc = LR_OK;
  for (int a = 0; a < 5; ++a) {
    const unsigned nb = (unsigned)((cnt[a] + 255) / 256);
    if (dtype == LR_F64)
      k_to_f64<double><<<nb, 256, 0, s>>>(static_cast<const double *>(src[a]), dk + off, (long long)cnt[a]);
    else
      k_to_f64<float><<<nb, 256, 0, s>>>(static_cast<const float *>(src[a]), dk + off, (long long)cnt[a]);
    off += cnt[a];
  }
  int hbits = 0;
  const size_t n = std::max(C, N);
  if (hipGetLastError() != hipSuccess || hipMemsetAsync(bits, 0, sizeof(int), s) != hipSuccess) {
    rc = set_err(c, LR_EDEVICE, "staging copy failed");
  } else {
    k_check_state<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
        nm, (int)C, (int)N, dk, dk + nm * C, dk + 2 * nm * C, dk + 3 * nm * C, dk + 3 * nm * C + N, bits);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&hbits, bits, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = set_err(c, LR_EDEVICE, "state check failed");
  }
  if (rc == LR_OK && (hbits & 1)) rc = set_err(c, LR_ENAN, "non-finite input");
  else if (rc == LR_OK && (hbits & 2))
    rc = set_err(c, LR_ESTATE, "volume fractions outside [0,1] or not summing to 1");
  else if (rc == LR_OK && (hbits & 4)) rc = set_err(c, LR_ESTATE, "rho <= 0 or e < 0 where k > 0");
  if (rc == LR_OK) rc = ctx_init_from_stage(c, t, dk);
  (void)hipStreamSynchronize(s);
  (void)hipFree(dk);
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
  return fp32(c) ? fields_out<float>(c->pf, buf, mask, out, c->outbuf, nullptr, c->stream, c->err)
                 : fields_out<double>(c->pd, buf, mask, out, c->outbuf, nullptr, c->stream, c->err);
}

int lr_totals(lr_ctx *c, double *out) {
  if (!c || !out) return LR_EINVAL;
  if (!c->have_state) return set_err(c, LR_ESTATE, "no state set");
  int rc = read_ctl(c);
  if (rc) return rc;
  const int buf = cur_slot(*c->hctl);
  return fp32(c) ? totals_out<float>(c->pf, buf, out, c->stream, c->err)
                 : totals_out<double>(c->pd, buf, out, c->stream, c->err);
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
    c->ev.resize((size_t)kChunk * 2 * kKernels);
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
