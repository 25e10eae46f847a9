// lr_batch.hpp — batch part of the C-ABI declared in include/lr.h (part of
// the lr_kernels.hip translation unit): many problems of different sizes in
// one device pool, stepped together by shared launches over the tiles of all
// running problems, admitted and retired between chunks of steps
// (continuous batching).
#pragma once

#include <deque>
#include <map>
#include <unordered_map>

namespace {

// First-fit ranges of one device pool; freed ranges merge with their
// neighbours.  Offsets and sizes are multiples of 256 bytes.
class PoolRanges {
 public:
  void init(size_t n) {
    free_.clear();
    if (n) free_[0] = n;
  }
  bool take(size_t n, size_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n, o = it->first;
      free_.erase(it);
      if (rest) free_[o + n] = rest;
      return true;
    }
    return false;
  }
  void give(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (const auto &f : free_) m = std::max(m, f.second);
    return m;
  }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
};

struct BatchReq {
  long id = -1;
  bool used = false, running = false;
  // admitted while a chunk was in flight: the chunk's copy of the control
  // records overwrites this slot's mirror with stale data, restored from ctl0
  bool fresh = false;
  Ctl ctl0{};
  int rc = LR_OK;
  size_t off = 0, bytes = 0;            // the problem's pool range
  size_t list_off = 0, list_bytes = 0;  // ... and its mixed-cell list's (grows)
  Grid g{};
  Prob<double> pd{};
  Prob<float> pf{};
};

}  // namespace

struct lr_batch {
  lr_batch_opts o{};
  hipStream_t own = nullptr, stream = nullptr;
  char *pool = nullptr;
  PoolRanges ranges;
  void *dprobs = nullptr;  // device Prob<R>[max_slots]
  size_t prob_size = 0;    // sizeof(Prob<R>)
  Ctl *ctl = nullptr;   // device [max_slots]
  Ctl *hctl = nullptr;  // pinned mirror, read after every chunk
  BlockMap *node_map = nullptr, *cell_map = nullptr;
  size_t node_cap = 0, cell_cap = 0;
  int node_blocks = 0, cell_blocks = 0;
  int *plist = nullptr;  // device [max_slots]: slots of the running problems
  int nprob = 0, mix_chunks = 16;
  bool maps_dirty = true;
  bool inflight = false;    // a chunk launched by lr_batch_step_begin, not yet ended
  bool chunk_timed = false;  // ... and timed for the autotuner
  long long chunk_cells = 0;
  StepFn step = nullptr;              // the step on the current tile shape
  StepFn steps[kTileShapes] = {};     // ... on each shape
  std::vector<BatchReq> slots;
  std::unordered_map<long, int> where;  // request id -> slot
  std::deque<long> finished;
  long next_id = 0;
  // input staging: a ring of pinned host and device buffers, each holding
  // one request's FP64 arrays until that request's set-up kernels ran; with
  // a chunk in flight, kStage admissions proceed without waiting for it
  static constexpr int kStage = 4;
  char *hstage[kStage] = {};
  double *dstage[kStage] = {};
  size_t stage_bytes[kStage] = {};
  hipEvent_t stage_ev[kStage] = {};
  int stage_next = 0;
  // outputs: copied on a stream of their own, so that the results of
  // finished requests come back while the next chunk runs
  hipStream_t io = nullptr;
  hipEvent_t io_wait = nullptr;
  std::vector<hipEvent_t> ready;  // per slot: recorded after its request's set-up kernels
  double *outbuf = nullptr;   // device
  size_t outbuf_n = 0;
  double *houtbuf = nullptr;  // pinned host
  size_t houtbuf_n = 0;
  hipGraphExec_t gexec = nullptr;
  bool graph_ok = false;
  // schedule autotuning: the first chunks run under each candidate schedule
  // (persistent grid x graph replay x tile shape), timed with events around
  // the launches, in one order and then the reverse
  static constexpr int kCand = LR_NSCHED;
  int tune_next = 0;               // next timing, 0 .. 2 kCand (done)
  double tune_ms[kCand] = {};      // time of the candidate's chunks
  double tune_work[kCand] = {};    // ... and their cell-steps
  double tune_rate[kCand] = {};    // cell-steps per ms
  hipEvent_t tune_ev[2] = {nullptr, nullptr};
  std::string err;
};

namespace {

int bset(lr_batch *b, int code, const std::string &msg) {
  if (b) b->err = msg;
  return code;
}
#define HIP_B(b, call)                                                                \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return bset((b), LR_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

bool bfp32(const lr_batch *b) { return b->o.precision == LR_FP32; }

size_t prob_bytes(const Grid &g, int precision) {
  if (precision == LR_FP32) {
    Prob<float> P;
    return carve_prob(P, nullptr, g, false, nullptr);
  }
  Prob<double> P;
  return carve_prob(P, nullptr, g, false, nullptr);
}
size_t list_bytes_of(const Grid &g, int precision, int cap) {
  return precision == LR_FP32 ? list_bytes<float>(g, cap) : list_bytes<double>(g, cap);
}

// request q (slot s) found more mixed cells than its list holds: a larger
// list from the pool, the descriptor on the device and the control record
// restored to the start of the step that stopped (see run_steps).  No pool
// range large enough: the request fails with LR_ENOMEM.
template <typename R>
int batch_list_grow(lr_batch *b, int s, BatchReq &q, Prob<R> &P) {
  Ctl &k = b->hctl[s];
  const int par = cur_slot(k);
  const int cap = mix_cap_grown(q.g, P.mix_cap, k.slot[par].nmix);
  const size_t nb = list_bytes<R>(q.g, cap);
  size_t off = 0;
  if (!b->ranges.take(nb, &off)) return LR_ENOMEM;
  b->ranges.give(q.list_off, q.list_bytes);  // no chunk is in flight: nothing reads it
  q.list_off = off;
  q.list_bytes = nb;
  carve_list(P, b->pool + off, q.g, cap);
  // chunks start at launch parity 0: the stopped step's slot becomes the
  // problem's parity-0 slot (the steps after it in the chunk did not count)
  P.flip = par;
  k.err = 0;
  k.slot[par].nmix = 0;
  k.slot[par].done = 0;
  HIP_B(b, hipMemcpyAsync(static_cast<char *>(b->dprobs) + s * b->prob_size, &P, sizeof(Prob<R>),
                          hipMemcpyHostToDevice, b->stream));
  HIP_B(b, hipMemcpyAsync(b->ctl + s, &k, sizeof(Ctl), hipMemcpyHostToDevice, b->stream));
  HIP_B(b, hipStreamSynchronize(b->stream));  // the host copies are read before they change
  return LR_OK;
}

// staging buffer r, free (its last request's set-up ran) and of `bytes` at least
int take_stage(lr_batch *b, int r, size_t bytes) {
  HIP_B(b, hipEventSynchronize(b->stage_ev[r]));
  if (bytes <= b->stage_bytes[r]) return LR_OK;
  const size_t n = std::max(bytes, b->stage_bytes[r] * 2);
  if (b->hstage[r]) (void)hipHostFree(b->hstage[r]);
  if (b->dstage[r]) (void)hipFree(b->dstage[r]);
  b->hstage[r] = nullptr;
  b->dstage[r] = nullptr;
  b->stage_bytes[r] = 0;
  if (hipHostMalloc((void **)&b->hstage[r], n, hipHostMallocDefault) != hipSuccess ||
      hipMalloc((void **)&b->dstage[r], n) != hipSuccess)
    return bset(b, LR_ENOMEM, "input staging");
  b->stage_bytes[r] = n;
  return LR_OK;
}

// output staging: n doubles on the device, nh pinned on the host
int grow_outbuf(lr_batch *b, size_t n, size_t nh) {
  if (n <= b->outbuf_n && nh <= b->houtbuf_n) return LR_OK;
  HIP_B(b, hipStreamSynchronize(b->io));
  if (n > b->outbuf_n) {
    if (b->outbuf) (void)hipFree(b->outbuf);
    b->outbuf = nullptr;
    b->outbuf_n = 0;
    if (hipMalloc((void **)&b->outbuf, n * sizeof(double)) != hipSuccess)
      return bset(b, LR_ENOMEM, "output staging");
    b->outbuf_n = n;
  }
  if (nh > b->houtbuf_n) {
    const size_t m = std::max(nh, 2 * b->houtbuf_n);
    if (b->houtbuf) (void)hipHostFree(b->houtbuf);
    b->houtbuf = nullptr;
    b->houtbuf_n = 0;
    if (hipHostMalloc((void **)&b->houtbuf, m * sizeof(double), hipHostMallocDefault) != hipSuccess)
      return bset(b, LR_ENOMEM, "output staging");
    b->houtbuf_n = m;
  }
  return LR_OK;
}

// block maps over the tiles of every running problem
int rebuild_maps(lr_batch *b) {
  std::vector<BlockMap> nm, cm;
  std::vector<int> pl;
  long long cmax = 0;
  for (size_t s = 0; s < b->slots.size(); ++s)
    if (b->slots[s].running) {
      tile_maps(b->slots[s].g, (int)s, nm, cm, kTileX[b->o.tile], kTileY[b->o.tile]);
      pl.push_back((int)s);
      cmax = std::max(cmax, (long long)b->slots[s].g.nx * b->slots[s].g.ny);
    }
  if (nm.size() > b->node_cap || cm.size() > b->cell_cap) {
    HIP_B(b, hipStreamSynchronize(b->stream));
    if (b->node_map) (void)hipFree(b->node_map);
    if (b->cell_map) (void)hipFree(b->cell_map);
    b->node_map = b->cell_map = nullptr;
    b->node_cap = std::max(nm.size(), 2 * b->node_cap);
    b->cell_cap = std::max(cm.size(), 2 * b->cell_cap);
    if (hipMalloc(&b->node_map, std::max<size_t>(b->node_cap, 1) * sizeof(BlockMap)) != hipSuccess ||
        hipMalloc(&b->cell_map, std::max<size_t>(b->cell_cap, 1) * sizeof(BlockMap)) != hipSuccess)
      return bset(b, LR_ENOMEM, "block maps");
  }
  // the maps are read by launches already queued: copy after they ran
  HIP_B(b, hipStreamSynchronize(b->stream));
  if (!nm.empty())
    HIP_B(b, hipMemcpy(b->node_map, nm.data(), nm.size() * sizeof(BlockMap), hipMemcpyHostToDevice));
  if (!cm.empty())
    HIP_B(b, hipMemcpy(b->cell_map, cm.data(), cm.size() * sizeof(BlockMap), hipMemcpyHostToDevice));
  if (!pl.empty()) HIP_B(b, hipMemcpy(b->plist, pl.data(), pl.size() * sizeof(int), hipMemcpyHostToDevice));
  b->node_blocks = (int)nm.size();
  b->cell_blocks = (int)cm.size();
  b->nprob = (int)pl.size();
  b->mix_chunks = mix_chunks_for(cmax, (int)pl.size());
  b->maps_dirty = false;
  b->graph_ok = false;
  return LR_OK;
}

template <typename R>
int batch_admit(lr_batch *b, int s, BatchReq &q, Prob<R> &P, const double *const in[5], double t_end,
                long long limit, int cap) {
  const Grid &g = q.g;
  const size_t C = (size_t)g.nx * g.ny, N = (size_t)(g.nx + 1) * (g.ny + 1), nm = g.nmat;
  carve_prob(P, b->pool + q.off, g, false, b->ctl + s);
  carve_list(P, b->pool + q.list_off, g, cap);
  int rc = clear_prob(P, b->stream, b->err);
  if (rc) return rc;
  const size_t nd = 3 * nm * C + 2 * N;
  const size_t bytes = nd * sizeof(double) + sizeof(Ctl) + sizeof(Prob<R>) + 512;
  const int r = b->stage_next;
  b->stage_next = (r + 1) % lr_batch::kStage;
  rc = take_stage(b, r, bytes);
  if (rc) return rc;
  double *hk = reinterpret_cast<double *>(b->hstage[r]);
  const size_t cnt[5] = {nm * C, nm * C, nm * C, N, N};
  size_t off = 0;
  for (int a = 0; a < 5; ++a) {
    std::memcpy(hk + off, in[a], cnt[a] * sizeof(double));
    off += cnt[a];
  }
  char *tail = b->hstage[r] + ((nd * sizeof(double) + 255) & ~size_t(255));
  Ctl *hc = reinterpret_cast<Ctl *>(tail);
  *hc = initial_ctl(0.0, t_end, limit);
  Prob<R> *hp = reinterpret_cast<Prob<R> *>(tail + ((sizeof(Ctl) + 255) & ~size_t(255)));
  *hp = P;
  b->hctl[s] = *hc;
  q.ctl0 = *hc;
  q.fresh = b->inflight;
  HIP_B(b, hipMemcpyAsync(b->dstage[r], hk, nd * sizeof(double), hipMemcpyHostToDevice, b->stream));
  HIP_B(b, hipMemcpyAsync(b->ctl + s, hc, sizeof(Ctl), hipMemcpyHostToDevice, b->stream));
  HIP_B(b, hipMemcpyAsync(static_cast<char *>(b->dprobs) + s * b->prob_size, hp, sizeof(Prob<R>),
                          hipMemcpyHostToDevice, b->stream));
  launch_init<R>(P, b->dstage[r], b->stream);
  HIP_B(b, hipGetLastError());
  HIP_B(b, hipEventRecord(b->stage_ev[r], b->stream));
  HIP_B(b, hipEventRecord(b->ready[s], b->stream));
  return LR_OK;
}

// run one chunk of steps of every running problem
int batch_chunk(lr_batch *b) {
  const Launch L{b->dprobs, b->node_map, b->cell_map, b->node_blocks, b->cell_blocks,
                 b->plist,  b->nprob,    b->mix_chunks, b->o.persistent != 0};
  const int n = b->o.chunk_steps;
  const bool timed = b->chunk_timed;
  if (!b->o.use_graph) {
    if (timed) HIP_B(b, hipEventRecord(b->tune_ev[0], b->stream));
    for (int st = 0; st < n; ++st) b->step(L, st & 1, b->stream, nullptr);
    HIP_B(b, hipGetLastError());
    if (timed) HIP_B(b, hipEventRecord(b->tune_ev[1], b->stream));
    return LR_OK;
  }
  if (!b->graph_ok) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    hipGraph_t graph = nullptr;
    HIP_B(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    for (int st = 0; st < n; ++st) b->step(L, st & 1, b->stream, nullptr);
    const hipError_t launch_err = hipGetLastError();
    const hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (launch_err != hipSuccess || e != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return bset(b, LR_EDEVICE, "graph capture failed");
    }
    const hipError_t ei = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return bset(b, LR_EDEVICE, "graph instantiation failed");
    b->graph_ok = true;
  }
  if (timed) HIP_B(b, hipEventRecord(b->tune_ev[0], b->stream));
  HIP_B(b, hipGraphLaunch(b->gexec, b->stream));
  if (timed) HIP_B(b, hipEventRecord(b->tune_ev[1], b->stream));
  return LR_OK;
}

// candidate schedule c: bit 0 persistent grid, bit 1 graph replay, c / 4
// the tile shape (whose block maps differ: rebuilt before the next chunk)
void set_schedule(lr_batch *b, int c) {
  const int pers = c & 1, graph = (c >> 1) & 1, tile = c >> 2;
  if (pers != b->o.persistent || graph != b->o.use_graph) b->graph_ok = false;
  if (tile != b->o.tile) b->maps_dirty = true;
  b->o.persistent = pers;
  b->o.use_graph = graph;
  b->o.tile = tile;
  b->step = b->steps[tile];
}
// the candidate of timing k: 0 .. kCand-1, then back down; a cost that
// drifts linearly over the tuning chunks adds the same to every candidate
int tune_candidate(int k) { return k < lr_batch::kCand ? k : 2 * lr_batch::kCand - 1 - k; }
bool tuning(const lr_batch *b) { return b->o.autotune && b->tune_next < 2 * lr_batch::kCand; }

// the output stream waits for the work on request q (slot s): a running
// request's, everything queued on the batch stream; another's, its set-up
// kernels (chunks that ran it were waited for when it finished)
int io_after(lr_batch *b, const BatchReq &q, int s) {
  if (q.running) {
    HIP_B(b, hipEventRecord(b->io_wait, b->stream));
    HIP_B(b, hipStreamWaitEvent(b->io, b->io_wait, 0));
  } else {
    HIP_B(b, hipStreamWaitEvent(b->io, b->ready[s], 0));
  }
  return LR_OK;
}

int find_req(lr_batch *b, long id, BatchReq **q) {
  auto it = b->where.find(id);
  if (it == b->where.end()) return bset(b, LR_EINVAL, "unknown request id");
  *q = &b->slots[it->second];
  return LR_OK;
}

}  // namespace

extern "C" {

void lr_batch_default_opts(lr_batch_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->max_slots = 256;
  o->pool_bytes = size_t(4) << 30;
  o->nmat = 2;
  o->precision = LR_FP32;
  o->chunk_steps = kChunk;
  o->use_graph = 1;
  o->persistent = 0;
  o->autotune = 0;
  o->tile = LR_TILE_32x8;
}

void lr_batch_destroy(lr_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->io) (void)hipStreamSynchronize(b->io);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  for (int r = 0; r < lr_batch::kStage; ++r) {
    if (b->stage_ev[r]) (void)hipEventDestroy(b->stage_ev[r]);
    if (b->dstage[r]) (void)hipFree(b->dstage[r]);
    if (b->hstage[r]) (void)hipHostFree(b->hstage[r]);
  }
  for (hipEvent_t e : b->ready)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : {b->tune_ev[0], b->tune_ev[1], b->io_wait})
    if (e) (void)hipEventDestroy(e);
  for (void *p : {(void *)b->pool, b->dprobs, (void *)b->ctl, (void *)b->node_map,
                  (void *)b->cell_map, (void *)b->outbuf, (void *)b->plist})
    if (p) (void)hipFree(p);
  if (b->hctl) (void)hipHostFree(b->hctl);
  if (b->houtbuf) (void)hipHostFree(b->houtbuf);
  if (b->io) (void)hipStreamDestroy(b->io);
  if (b->own) (void)hipStreamDestroy(b->own);
  delete b;
}

int lr_batch_create(const lr_batch_opts *opts, lr_batch **out) {
  if (!out) return LR_EINVAL;
  *out = nullptr;
  lr_batch_opts o;
  if (opts) o = *opts;
  else lr_batch_default_opts(&o);
  if (o.max_slots < 1 || o.max_slots > (1 << 20) || o.pool_bytes < 256 || o.nmat < 1 ||
      o.nmat > LR_MAXMAT || (o.precision != LR_FP64 && o.precision != LR_FP32) ||
      o.chunk_steps < 2 || (o.chunk_steps & 1) || o.tile < 0 || o.tile >= LR_NTILE)
    return LR_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return LR_EDEVICE;
  lr_batch *b = new (std::nothrow) lr_batch();
  if (!b) return LR_ENOMEM;
  b->o = o;
  b->o.pool_bytes &= ~size_t(255);
  // the kernels index the descriptors as an array of Prob<R>
  b->prob_size = o.precision == LR_FP32 ? sizeof(Prob<float>) : sizeof(Prob<double>);
  b->slots.resize(o.max_slots);
  int rc = LR_OK;
  if (hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&b->io, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->io_wait, hipEventDisableTiming) != hipSuccess ||
      hipEventCreate(&b->tune_ev[0]) != hipSuccess || hipEventCreate(&b->tune_ev[1]) != hipSuccess)
    rc = LR_EDEVICE;
  for (int r = 0; rc == LR_OK && r < lr_batch::kStage; ++r)
    if (hipEventCreateWithFlags(&b->stage_ev[r], hipEventDisableTiming) != hipSuccess) rc = LR_EDEVICE;
  b->ready.assign(o.max_slots, nullptr);
  for (int s = 0; rc == LR_OK && s < o.max_slots; ++s)
    if (hipEventCreateWithFlags(&b->ready[s], hipEventDisableTiming) != hipSuccess) rc = LR_EDEVICE;
  b->stream = b->own;
  if (rc == LR_OK && (hipMalloc((void **)&b->pool, b->o.pool_bytes) != hipSuccess ||
                      hipMalloc(&b->dprobs, b->prob_size * o.max_slots) != hipSuccess ||
                      hipMalloc((void **)&b->ctl, sizeof(Ctl) * o.max_slots) != hipSuccess ||
                      hipMalloc((void **)&b->plist, sizeof(int) * o.max_slots) != hipSuccess ||
                      hipHostMalloc((void **)&b->hctl, sizeof(Ctl) * o.max_slots, hipHostMallocDefault) !=
                          hipSuccess))
    rc = LR_ENOMEM;
  if (rc == LR_OK) {
    std::memset(b->hctl, 0, sizeof(Ctl) * o.max_slots);
    b->ranges.init(b->o.pool_bytes);
    // every shape's step, its resident block counts queried before any capture
    for (int t = 0; t < kTileShapes; ++t)
      b->steps[t] = bfp32(b) ? step_fn_tile<float>(o.nmat, t) : step_fn_tile<double>(o.nmat, t);
    b->step = b->steps[o.tile];
    // every event recorded once, so that waiting on one never waits on nothing
    for (int r = 0; rc == LR_OK && r < lr_batch::kStage; ++r)
      if (hipEventRecord(b->stage_ev[r], b->stream) != hipSuccess) rc = LR_EDEVICE;
    // staging and output buffers for requests up to about 128 x 128 cells,
    // allocated now: an allocation while a chunk is in flight can wait for it
    for (int r = 0; rc == LR_OK && r < lr_batch::kStage; ++r) rc = take_stage(b, r, size_t(1) << 20);
    if (rc == LR_OK) rc = grow_outbuf(b, size_t(1) << 17, size_t(1) << 17);
    for (int s = 0; rc == LR_OK && s < o.max_slots; ++s)
      if (hipEventRecord(b->ready[s], b->stream) != hipSuccess) rc = LR_EDEVICE;
  }
  if (rc != LR_OK) {
    lr_batch_destroy(b);
    return rc;
  }
  *out = b;
  return LR_OK;
}

int lr_batch_bind_stream(lr_batch *b, void *hip_stream) {
  if (!b) return LR_EINVAL;
  if (b->inflight) return bset(b, LR_EINVAL, "a chunk is in flight: end it first");
  HIP_B(b, hipStreamSynchronize(b->stream));
  b->stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : b->own;
  return LR_OK;
}

size_t lr_batch_footprint(int nx, int ny, int nmat, int precision) {
  if (nx < 2 || ny < 2 || nmat < 1 || nmat > LR_MAXMAT) return 0;
  Grid g{};
  g.nx = nx;
  g.ny = ny;
  g.nmat = nmat;
  return prob_bytes(g, precision) + list_bytes_of(g, precision, mix_cap_initial(g, 0));
}

int lr_batch_submit(lr_batch *b, int nx, int ny, const lr_eos *eos, const lr_opts *opts, double t_end,
                    long max_steps, const double *k, const double *rho, const double *e,
                    const double *ux, const double *uy, long *req_id) {
  if (!b || !req_id || !k || !rho || !e || !ux || !uy) return LR_EINVAL;
  *req_id = -1;
  lr_opts o;
  if (opts) o = *opts;
  else {
    lr_default_opts(&o);
    o.precision = b->o.precision;
  }
  if (o.precision != b->o.precision || o.stages || o.remap != LR_REMAP_DIRECTCF)
    return bset(b, LR_EINVAL, "precision differs from the batch's, or stages or the AD remap set");
  if (!(t_end >= 0.0) || max_steps < 0) return bset(b, LR_EINVAL, "t_end < 0 or max_steps < 0");
  Grid g;
  if (make_grid(nx, ny, b->o.nmat, eos, nullptr, o, g) != LR_OK) return bset(b, LR_EINVAL, "bad grid, eos or options");
  const char *msg = "";
  const int chk = check_state_host(g, k, rho, e, ux, uy, &msg);
  if (chk) return bset(b, chk, msg);
  int s = -1;
  for (int i = 0; i < (int)b->slots.size(); ++i)
    if (!b->slots[i].used) {
      s = i;
      break;
    }
  if (s < 0) return bset(b, LR_EAGAIN, "no free slot");
  const size_t bytes = prob_bytes(g, b->o.precision);
  const int cap = mix_cap_initial(g, count_mixed_host(g, k));
  const size_t lbytes = list_bytes_of(g, b->o.precision, cap);
  size_t off = 0, loff = 0;
  if (!b->ranges.take(bytes, &off)) return bset(b, LR_EAGAIN, "no pool range large enough");
  if (!b->ranges.take(lbytes, &loff)) {
    b->ranges.give(off, bytes);
    return bset(b, LR_EAGAIN, "no pool range large enough");
  }
  BatchReq &q = b->slots[s];
  q = BatchReq{};
  q.g = g;
  q.off = off;
  q.bytes = bytes;
  q.list_off = loff;
  q.list_bytes = lbytes;
  const double *in[5] = {k, rho, e, ux, uy};
  const int rc = bfp32(b) ? batch_admit<float>(b, s, q, q.pf, in, t_end, max_steps, cap)
                          : batch_admit<double>(b, s, q, q.pd, in, t_end, max_steps, cap);
  if (rc != LR_OK) {
    b->ranges.give(off, bytes);
    b->ranges.give(loff, lbytes);
    q = BatchReq{};
    return rc;
  }
  q.used = true;
  q.id = b->next_id++;
  b->where[q.id] = s;
  const Slot &s0 = q.ctl0.slot[0];
  if (s0.done) {
    b->finished.push_back(q.id);
  } else {
    q.running = true;
    b->maps_dirty = true;
  }
  *req_id = q.id;
  return LR_OK;
}

int lr_batch_step_begin(lr_batch *b) {
  if (!b) return LR_EINVAL;
  if (b->inflight) return bset(b, LR_EINVAL, "a chunk is already in flight");
  int rc = LR_OK;
  b->chunk_timed = tuning(b);
  if (b->chunk_timed) set_schedule(b, tune_candidate(b->tune_next));
  if (b->maps_dirty) rc = rebuild_maps(b);
  if (rc) return rc;
  if (b->node_blocks == 0) return LR_OK;  // nothing runs; the end call only counts
  b->chunk_cells = 0;
  if (b->chunk_timed)
    for (const auto &q : b->slots)
      if (q.running) b->chunk_cells += (long long)q.g.nx * q.g.ny;
  rc = batch_chunk(b);
  if (rc) return rc;
  HIP_B(b, hipMemcpyAsync(b->hctl, b->ctl, sizeof(Ctl) * b->slots.size(), hipMemcpyDeviceToHost,
                          b->stream));
  b->inflight = true;
  return LR_OK;
}

int lr_batch_step_end(lr_batch *b, int *n_running) {
  if (!b) return LR_EINVAL;
  int running = 0;
  if (!b->inflight) {
    for (const auto &q : b->slots) running += q.running;
    if (n_running) *n_running = running;
    return LR_OK;
  }
  b->inflight = false;
  HIP_B(b, hipStreamSynchronize(b->stream));
  for (size_t s = 0; s < b->slots.size(); ++s) {
    BatchReq &q = b->slots[s];
    if (q.used && q.fresh) {
      b->hctl[s] = q.ctl0;
      q.fresh = false;
    }
  }
  if (b->chunk_timed) {
    float ms = 0.0f;
    HIP_B(b, hipEventElapsedTime(&ms, b->tune_ev[0], b->tune_ev[1]));
    const int c = tune_candidate(b->tune_next);
    b->tune_ms[c] += ms;
    b->tune_work[c] += double(b->chunk_cells) * b->o.chunk_steps;
    if (++b->tune_next == 2 * lr_batch::kCand) {
      int best = 0;
      for (int k = 0; k < lr_batch::kCand; ++k) {
        b->tune_rate[k] = b->tune_ms[k] > 0.0 ? b->tune_work[k] / b->tune_ms[k] : 0.0;
        if (b->tune_rate[k] > b->tune_rate[best]) best = k;
      }
      set_schedule(b, best);
    }
  }
  for (size_t s = 0; s < b->slots.size(); ++s) {
    BatchReq &q = b->slots[s];
    if (!q.running) continue;
    const Ctl &k = b->hctl[s];
    if (k.err == ERR_MIXCAP) {  // a step stopped for a larger list: grow it, the request goes on
      const int rg = bfp32(b) ? batch_list_grow<float>(b, (int)s, q, q.pf)
                              : batch_list_grow<double>(b, (int)s, q, q.pd);
      if (rg == LR_OK) {
        ++running;
        continue;
      }
      if (rg != LR_ENOMEM) return rg;
    }
    if (k.slot[cur_slot(k)].done || k.err) {
      const char *msg = "";
      q.rc = err_code(k.err, &msg);
      q.running = false;
      b->finished.push_back(q.id);
      b->maps_dirty = true;
    } else {
      ++running;
    }
  }
  if (n_running) *n_running = running;
  return LR_OK;
}

int lr_batch_step(lr_batch *b, int *n_running) {
  const int rc = lr_batch_step_begin(b);
  if (rc) return rc;
  return lr_batch_step_end(b, n_running);
}

int lr_batch_running(lr_batch *b) {
  if (!b) return 0;
  int n = 0;
  for (const auto &q : b->slots) n += q.running;
  return n;
}

int lr_batch_poll(lr_batch *b, long *ids, int cap, int *n) {
  if (!b || !n || cap < 0 || (cap > 0 && !ids)) return LR_EINVAL;
  int m = 0;
  while (m < cap && !b->finished.empty()) {
    ids[m++] = b->finished.front();
    b->finished.pop_front();
  }
  *n = m;
  return LR_OK;
}

int lr_batch_status(lr_batch *b, long id, int *rc, long *steps, double *t) {
  if (!b) return LR_EINVAL;
  BatchReq *q = nullptr;
  const int r = find_req(b, id, &q);
  if (r) return r;
  const int s = b->where[id];
  const Ctl &k = b->hctl[s];
  const Slot &cur = k.slot[cur_slot(k)];
  if (rc) *rc = q->running ? LR_EAGAIN : q->rc;
  if (steps) *steps = (long)cur.step;
  if (t) *t = cur.t;
  return LR_OK;
}

int lr_batch_get_fields(lr_batch *b, long id, unsigned mask, double *const *out) {
  if (!b || !out) return LR_EINVAL;
  BatchReq *q = nullptr;
  int rc = find_req(b, id, &q);
  if (rc) return rc;
  const Grid &g = q->g;
  size_t nh = 0;
  for (unsigned bit = 1; bit <= LR_F_IE; bit <<= 1)
    if (mask & bit) nh += field_count(g, bit);
  rc = grow_outbuf(b, std::max((size_t)g.nmat * g.nx * g.ny, (size_t)(g.nx + 1) * (g.ny + 1)), nh);
  if (rc) return rc;
  const int s = b->where[id];
  const int buf = cur_slot(b->hctl[s]);
  rc = io_after(b, *q, s);
  if (rc) return rc;
  return bfp32(b) ? fields_out<float>(q->pf, buf, mask, out, b->outbuf, b->houtbuf, b->io, b->err)
                  : fields_out<double>(q->pd, buf, mask, out, b->outbuf, b->houtbuf, b->io, b->err);
}

int lr_batch_totals(lr_batch *b, long id, double *out) {
  if (!b || !out) return LR_EINVAL;
  BatchReq *q = nullptr;
  const int rc = find_req(b, id, &q);
  if (rc) return rc;
  const int s = b->where[id];
  const int buf = cur_slot(b->hctl[s]);
  const int rw = io_after(b, *q, s);
  if (rw) return rw;
  return bfp32(b) ? totals_out<float>(q->pf, buf, out, b->io, b->err)
                  : totals_out<double>(q->pd, buf, out, b->io, b->err);
}

int lr_batch_release(lr_batch *b, long id) {
  if (!b) return LR_EINVAL;
  BatchReq *q = nullptr;
  const int rc = find_req(b, id, &q);
  if (rc) return rc;
  // launches still queued may read a running problem: free its range after
  // them.  A request that is not running is in no queued launch, and its
  // set-up kernels are ahead of any later admission's on the batch stream.
  if (q->running) {
    HIP_B(b, hipStreamSynchronize(b->stream));
    b->maps_dirty = true;
  }
  b->ranges.give(q->off, q->bytes);
  b->ranges.give(q->list_off, q->list_bytes);
  b->where.erase(id);
  *q = BatchReq{};
  return LR_OK;
}

int lr_batch_schedule(lr_batch *b, int *persistent, int *use_graph, int *tile, double *rates) {
  if (!b) return LR_EINVAL;
  if (persistent) *persistent = b->o.persistent;
  if (use_graph) *use_graph = b->o.use_graph;
  if (tile) *tile = b->o.tile;
  if (rates)
    for (int c = 0; c < lr_batch::kCand; ++c) rates[c] = b->tune_rate[c];
  return tuning(b) ? LR_EAGAIN : LR_OK;
}

const char *lr_batch_last_error(const lr_batch *b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
