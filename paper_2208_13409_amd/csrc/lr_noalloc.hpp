// lr_noalloc.hpp — the allocation-free entry point lr_run_noalloc (part of
// the lr_kernels.hip translation unit).  One call sets up a problem from
// device inputs, steps it and writes the requested fields to device outputs,
// with every device array the step kernels need (state, transients, control
// record, descriptor, block maps) carved from `scratch`, a file-scope device
// array of LR_NOALLOC_BYTES bytes.  It calls no hipMalloc, hipFree or other
// allocating routine, for callers that cannot allocate.
#pragma once

#include <mutex>

namespace {

// The workspace.  Each device the library runs on holds its own copy until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: host code only ever uses the address hipGetSymbolAddress
// returns for the current device (noalloc_base).
__device__ __align__(256) char scratch[LR_NOALLOC_BYTES];

constexpr int kNoallocDevices = 64;
std::mutex g_noalloc_mu;
char *g_noalloc_ptr[kNoallocDevices] = {nullptr};

// Errors of this path go to a fixed buffer: nothing here allocates, on the
// device or on the host.
struct NoallocErr {
  char m[256];
  int set(int code, const char *a, const char *b = "") {
    std::snprintf(m, sizeof m, "%s%s", a, b);
    return code;
  }
};
#define NA_TRY(err, call)                                                  \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess) return (err).set(LR_EDEVICE, #call ": ", hipGetErrorString(e_)); \
  } while (0)

// the device address of the current device's workspace, looked up once per
// device with that device current
int noalloc_base(char **out, NoallocErr &err) {
  int dev = 0;
  NA_TRY(err, hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoallocDevices) return err.set(LR_EDEVICE, "device index beyond the workspace table");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *p = nullptr;
    NA_TRY(err, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return err.set(LR_EDEVICE, "hipGetSymbolAddress gave a null workspace address");
    g_noalloc_ptr[dev] = static_cast<char *>(p);
  }
  *out = g_noalloc_ptr[dev];
  return LR_OK;
}

// the control record of a fresh state at time t (initial_ctl(t, t, 0)),
// written on the device: the record is larger than a kernel's arguments
__global__ void k_noalloc_ctl(Ctl *ctl, double t) {
  const int i = threadIdx.x;
  const unsigned long long inf = 0x7ff0000000000000ull;  // bits of +inf
  for (int s = 0; s < 2; ++s)
    for (int k = i; k < NDT; k += blockDim.x) ctl->slot[s].dtmin[k] = inf;
  if (i == 0) {
    for (int s = 0; s < 2; ++s) {
      Slot &sl = ctl->slot[s];
      sl.t = t;
      sl.t_end = t;
      sl.step = s == 0 ? 0 : -1;
      sl.limit = 0;
      sl.done = 1;
      sl.nmix = 0;
    }
    ctl->err = 0;
    ctl->pad = 0;
  }
}

// the problem descriptor, the problem list {0} of the mixed-cell launch, a
// cleared check word, and the block maps in the order tile_maps lists them
// (node tiles over [0, nx] x [0, ny], cell tiles over [0, nx) x [0, ny))
template <typename R>
__global__ void k_noalloc_setup(Prob<R> P, Prob<R> *dprob, int *plist, int *bits, BlockMap *node_map,
                                int node_blocks, BlockMap *cell_map, int cell_blocks) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int nx = P.g.nx, ny = P.g.ny;
  if (b == 0) {
    *dprob = P;
    *plist = 0;
    *bits = 0;
  }
  constexpr int TX = TileDefault::TX, TY = TileDefault::TY;
  const int nbx = nx / TX + 1, cbx = (nx + TX - 1) / TX;
  if (b < node_blocks) node_map[b] = BlockMap{0, (b % nbx) * TX, (b / nbx) * TY, 0};
  if (b < cell_blocks) cell_map[b] = BlockMap{0, (b % cbx) * TX, (b / cbx) * TY, 0};
}

struct NoallocArgs {
  double t0, t_end;
  long max_steps;
  const double *k, *rho, *e, *ux, *uy;
  unsigned mask;
  double *const *out;
  hipStream_t s;
  long steps;
  double t;
};

template <typename R>
int noalloc_run(const Grid &g, char *base, NoallocArgs &a, NoallocErr &err) {
  const size_t C = (size_t)g.nx * g.ny, N = (size_t)(g.nx + 1) * (g.ny + 1);
  constexpr int TX = TileDefault::TX, TY = TileDefault::TY;
  const int node_blocks = (g.nx / TX + 1) * (g.ny / TY + 1);
  const int cell_blocks = ((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY);
  // layout: control record, descriptor, problem list, check word, block
  // maps, the problem's arrays as lr_create carves them, then the list of
  // mixed cells, as long as the rest of the workspace allows (up to one
  // entry per cell; it cannot grow here)
  Carver cv{nullptr};
  cv.take<Ctl>(1);
  cv.take<Prob<R>>(1);
  cv.take<int>(1);
  cv.take<int>(1);
  cv.take<BlockMap>(node_blocks);
  cv.take<BlockMap>(cell_blocks);
  const size_t head = (cv.off + 255) & ~size_t(255);
  Prob<R> P;
  const size_t body = carve_prob(P, nullptr, g, false, nullptr);
  const int cap_min = mix_cap_initial(g, 0);
  const size_t need = head + body + list_bytes<R>(g, cap_min);
  if (need > (size_t)LR_NOALLOC_BYTES) {
    std::snprintf(err.m, sizeof err.m, "problem needs %zu bytes of device memory; the static workspace holds %zu",
                  need, (size_t)LR_NOALLOC_BYTES);
    return LR_ENOMEM;
  }
  // the largest list that fits, one entry per cell at most
  const size_t entry = sizeof(int) + 8 * (size_t)g.nmat * sizeof(R);
  const size_t room = (size_t)LR_NOALLOC_BYTES - head - body - 512;
  const int cap = (int)std::min<size_t>(C, std::max<size_t>(cap_min, room / entry));
  cv = Carver{base};
  Ctl *ctl = cv.take<Ctl>(1);
  Prob<R> *dprob = cv.take<Prob<R>>(1);
  int *plist = cv.take<int>(1);
  int *bits = cv.take<int>(1);
  BlockMap *node_map = cv.take<BlockMap>(node_blocks);
  BlockMap *cell_map = cv.take<BlockMap>(cell_blocks);
  carve_prob(P, base + head, g, false, ctl);
  carve_list(P, base + head + body, g, cap);
  if (head + body + list_bytes<R>(g, cap) > (size_t)LR_NOALLOC_BYTES) {
    std::snprintf(err.m, sizeof err.m, "mixed-cell list does not fit the workspace");
    return LR_ENOMEM;
  }
  hipStream_t s = a.s;

  // descriptor, maps, control record; wall flux entries cleared (the
  // workspace keeps whatever the previous call left)
  const int nb = std::max(node_blocks, cell_blocks);
  k_noalloc_setup<R><<<(unsigned)((nb + 255) / 256), 256, 0, s>>>(P, dprob, plist, bits, node_map, node_blocks,
                                                                  cell_map, cell_blocks);
  k_noalloc_ctl<<<1, 256, 0, s>>>(ctl, a.t0);
  NA_TRY(err, hipGetLastError());
  const size_t nX = (size_t)(g.nx + 1) * g.ny, nY = (size_t)g.nx * (g.ny + 1);
  NA_TRY(err, hipMemsetAsync(P.MX, 0, nX * sizeof(R), s));
  NA_TRY(err, hipMemsetAsync(P.MY, 0, nY * sizeof(R), s));
  NA_TRY(err, hipMemsetAsync(P.MC, 0, N * sizeof(R), s));

  // the checks of lr_set_state on the device inputs
  const size_t n = std::max(C, N);
  k_check_state<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g.nmat, (int)C, (int)N, a.k, a.rho, a.e, a.ux,
                                                            a.uy, bits);
  NA_TRY(err, hipGetLastError());
  int hbits = 0;
  NA_TRY(err, hipMemcpyAsync(&hbits, bits, sizeof(int), hipMemcpyDeviceToHost, s));
  NA_TRY(err, hipStreamSynchronize(s));
  if (hbits & 1) return err.set(LR_ENAN, "non-finite input");
  if (hbits & 2) return err.set(LR_ESTATE, "volume fractions outside [0,1] or not summing to 1");
  if (hbits & 4) return err.set(LR_ESTATE, "rho <= 0 or e < 0 where k > 0");

  // initial state, sound speed and the first CFL bound (as lr_set_state)
  const unsigned cb = (unsigned)((C + 255) / 256), nbk = (unsigned)((N + 255) / 256);
  k_init_state<R><<<cb, 256, 0, s>>>(P, a.k, a.rho, a.e);
  k_init_vel<R><<<nbk, 256, 0, s>>>(P, a.ux, a.uy);
  k_sound<R><<<cb, 256, 0, s>>>(P, 0);
  k_dt_bound<R><<<nbk, 256, 0, s>>>(P, 0);
  k_start<<<1, 1, 0, s>>>(ctl, a.t_end, (long long)a.max_steps);
  NA_TRY(err, hipGetLastError());

  // steps in chunks, the host reading the control record between chunks
  // (as lr_run)
  const Launch L{dprob, node_map, cell_map, node_blocks, cell_blocks, plist, 1,
                 mix_chunks_for((long long)C), false};
  const StepFn step = step_fn<R>(g.nmat);
  Ctl h;
  int gpar = 0;
  for (;;) {
    NA_TRY(err, hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    NA_TRY(err, hipStreamSynchronize(s));
    const Slot &sl = h.slot[cur_slot(h)];
    if (sl.done || h.err) break;
    const long long left = sl.limit - sl.step;
    const long long nst = left < kChunk ? left : kChunk;
    for (long long st = 0; st < nst; ++st) {
      step(L, gpar, s, nullptr);
      gpar ^= 1;
    }
    NA_TRY(err, hipGetLastError());
  }
  const int cur = cur_slot(h);
  a.steps = (long)h.slot[cur].step;
  a.t = h.slot[cur].t;
  if (h.err) {
    const char *msg = "";
    const int rc = err_code(h.err, &msg);
    return err.set(rc, msg);
  }

  // fields of the final state straight into the caller's device arrays
  int slot = 0;
  for (unsigned bit = 1; bit <= LR_F_IE; bit <<= 1) {
    if (!(a.mask & bit)) continue;
    double *o = a.out[slot++];
    if (!o) return err.set(LR_EINVAL, "null output pointer");
    k_fields<R><<<nbk, 256, 0, s>>>(P, cur, bit, o);
  }
  NA_TRY(err, hipGetLastError());
  NA_TRY(err, hipStreamSynchronize(s));
  return LR_OK;
}

void noalloc_msg(char *buf, size_t len, const char *m) {
  if (buf && len) std::snprintf(buf, len, "%s", m);
}

}  // namespace

extern "C" int lr_run_noalloc(int nx, int ny, int nmat, const lr_eos *eos, const int bc[4],
                              const lr_opts *opts, double t0, double t_end, long max_steps,
                              const double *k, const double *rho, const double *e, const double *ux,
                              const double *uy, unsigned field_mask, double *const *out, void *hip_stream,
                              long *steps_out, double *t_out, char *errbuf, size_t errlen) {
  NoallocErr err;
  err.m[0] = '\0';
  noalloc_msg(errbuf, errlen, "");
  lr_opts o;
  if (opts) o = *opts;
  else lr_default_opts(&o);
  Grid g;
  if (make_grid(nx, ny, nmat, eos, bc, o, g) != LR_OK) {
    noalloc_msg(errbuf, errlen, "invalid grid, materials or options");
    return LR_EINVAL;
  }
  if (o.stages || o.remap != LR_REMAP_DIRECTCF) {
    noalloc_msg(errbuf, errlen, "opts.stages must be 0 and opts.remap LR_REMAP_DIRECTCF");
    return LR_EINVAL;
  }
  if (!k || !rho || !e || !ux || !uy || (field_mask && !out) || field_mask > 2 * LR_F_IE - 1 ||
      !std::isfinite(t0) || !(t_end >= t0) || max_steps < 0) {
    noalloc_msg(errbuf, errlen, "null input, bad field mask, t_end < t0 or max_steps < 0");
    return LR_EINVAL;
  }
  char *base = nullptr;
  int rc = noalloc_base(&base, err);
  if (rc == LR_OK) {
    NoallocArgs a{t0, t_end, max_steps, k, rho, e, ux, uy, field_mask, out,
                  static_cast<hipStream_t>(hip_stream), 0, t0};
    rc = o.precision == LR_FP32 ? noalloc_run<float>(g, base, a, err) : noalloc_run<double>(g, base, a, err);
    if (steps_out) *steps_out = a.steps;
    if (t_out) *t_out = a.t;
  }
  if (rc != LR_OK) noalloc_msg(errbuf, errlen, err.m);
  return rc;
}
