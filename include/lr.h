/*
 * lr.h — C-ABI of the MI355X library for the 2D multimaterial Lagrange–Remap
 * step with the one-step "Direct remap with Corner Fluxes" (DirectCF) of
 * B. Chaudet, arXiv:2208.13409.  One context holds one problem: a regular
 * orthogonal grid of nx x ny cells, nmat perfect-gas or stiffened-gas
 * materials and reflective walls.  All state lives in device memory owned by the library; every
 * argument pointer below is HOST memory, FP64, row-major with x fastest,
 * unless stated otherwise.
 *
 * Every function returns 0 (LR_OK) or a negative LR_E* code and never aborts;
 * lr_last_error() then describes the failure.  A context is not thread-safe:
 * one host thread at a time per context.  Kernels run on the context's HIP
 * stream (its own non-blocking stream unless lr_bind_stream is called).
 */
#ifndef LR_H
#define LR_H
#include <stddef.h>
#ifdef __cplusplus
extern "C" {
#endif

#define LR_MAXMAT 4

enum {
  LR_OK = 0,
  LR_EINVAL = -1,    /* bad argument (sizes, options, null pointers, t_end < t) */
  LR_ENOMEM = -2,    /* device or host allocation failed                        */
  LR_EDEVICE = -3,   /* a HIP call failed                                       */
  LR_ENEGATIVE = -4, /* negative partial volume / mass / energy, Vol^lagCF <= 0 */
  LR_ENAN = -5,      /* non-finite value in the inputs or the state             */
  LR_EDT = -6,       /* time step not positive or not finite                    */
  LR_EAGAIN = -7,    /* a batch has no free slot or device memory for it now    */
  LR_ESTATE = -8     /* no state set, or volume fractions outside [0,1] / sum != 1 */
};

enum { LR_BC_REFLECT = 0 };     /* the only boundary: reflective wall          */
enum { LR_FP64 = 0, LR_FP32 = 1 };
/* remap of the Lagrangian state: the one-step DirectCF remap with corner
 * fluxes (§2.3, the default), or the paper's comparator, the alternate-
 * direction remap (§2.1.1, §2.1.2, §4.2): an X pass then a Y pass, in the
 * other order on every second step, each a one-dimensional remap of the cell
 * and nodal quantities with its own interface */
enum { LR_REMAP_DIRECTCF = 0, LR_REMAP_AD = 1 };

/* material equation of state p = (gamma-1) rho e - pinf: the perfect gas of
 * paper §5.1 for pinf = 0, the stiffened gas of §5.2 (the paper's pi, e.g.
 * water gamma 7, pi 2.1e9 Pa) for pinf > 0; gamma > 1, pinf >= 0 and finite.
 * The squared sound speed is (gamma p + pinf) / rho. */
typedef struct { double gamma, pinf; } lr_eos;

typedef struct {
  double x0, x1, y0, y1; /* domain; dx = (x1-x0)/nx, dy = (y1-y0)/ny                    */
  double cfl;            /* CFL number; default 0.5                                     */
  double a1, a2;         /* Wilkins linear / quadratic pseudo-viscosity (§1.2); 0.5, 1.0  */
  int precision;         /* LR_FP64 (default) or LR_FP32: FP32 bulk arithmetic and state,
                            FP64 interface, clipping and totals, compensated cell sums    */
  int recon_order;       /* 1 = upwind everywhere, 2 = limited linear along each region's
                            direction (§2.1.1, §3.3), 3 = the multidimensional least-
                            squares plane of §3.3 for the cell quantities (DirectCF only;
                            the nodal velocities keep order 2)                           */
  int kinematic;         /* 1 = node velocities prescribed, no forces, no momentum remap  */
  double k_eps;          /* a material is present where V_a > k_eps * dx*dy; 1e-10
                            (FP32 uses at least 1e-6)                                     */
  double fixed_dt;       /* > 0: this time step instead of the CFL one                    */
  int stages;            /* 1 = keep the intermediates of each step for lr_debug_get      */
  int remap;             /* LR_REMAP_DIRECTCF (default) or LR_REMAP_AD; batches and
                            lr_run_noalloc run DirectCF only                              */
  int mix_list;          /* initial capacity (cells) of the list of mixed cells; 0
                            (default): the larger of nx*ny/16, 256 and twice the mixed
                            cells of the initial state.  A step that finds more mixed
                            cells stops before it changes the state; the list grows
                            and the step runs again (lr_run_noalloc: the largest list
                            its workspace holds, no growth)                              */
  int tile;              /* tile shape of a context's step kernels (LR_TILE_*, below):
                            LR_TILE_AUTO (default) counts the grid's node tiles against
                            the device's CUs: 32x8 if its 32x8 tiles fit one block per
                            CU, else 32x12 if those do (one latency-bound round instead
                            of two blocks on some CUs), else 32x16.  LR_REMAP_AD runs
                            on 32x8 only; batches take their shape from lr_batch_opts
                            and lr_run_noalloc runs 32x8.  Results do not depend on it. */
} lr_opts;

/* field mask bits for lr_get_fields, in the order the output pointers are
 * given (lowest bit first).  Mixture fields are [ny][nx]; per-material fields
 * [nmat][ny][nx] (0 where the material is absent); node fields [ny+1][nx+1]. */
enum {
  LR_F_RHO = 1,      /* mixture density  sum M_a / (dx dy)                    */
  LR_F_P = 2,        /* mixture pressure sum k_a P_a (§4.1)                   */
  LR_F_E = 4,        /* mixture specific internal energy sum E_a / sum M_a    */
  LR_F_K = 8,        /* volume fractions V_a / (dx dy)                        */
  LR_F_RHOA = 16,    /* partial densities M_a / V_a                           */
  LR_F_EA = 32,      /* partial specific internal energies E_a / M_a          */
  LR_F_PA = 64,      /* partial pressures                                     */
  LR_F_UX = 128,     /* nodal velocity x                                      */
  LR_F_UY = 256,     /* nodal velocity y                                      */
  LR_F_VOL = 512,    /* conserved partial volumes V_a                         */
  LR_F_MASS = 1024,  /* conserved partial masses M_a                          */
  LR_F_IE = 2048     /* conserved partial internal energies E_a = M_a e_a     */
};

typedef struct lr_ctx lr_ctx;

/* fill *o with the defaults listed in lr_opts */
void lr_default_opts(lr_opts *o);

/* Create a problem context and allocate its device memory on the current HIP
 * device.  nx, ny >= 2, nx*ny <= 2^28 (32-bit cell indices with up to
 * LR_MAXMAT materials); 1 <= nmat <= LR_MAXMAT; eos[nmat]; bc[4] = {xlo, xhi,
 * ylo, yhi}, all LR_BC_REFLECT (NULL means all reflective); opts NULL means
 * defaults.  *out receives the context (NULL on failure). */
int lr_create(int nx, int ny, int nmat, const lr_eos *eos, const int bc[4],
              const lr_opts *opts, lr_ctx **out);

/* Launch this context's kernels on the given hipStream_t (passed as void*,
 * e.g. torch.cuda.current_stream().cuda_stream).  The caller keeps the
 * stream alive; NULL returns to the context's own stream. */
int lr_bind_stream(lr_ctx *c, void *hip_stream);

/* Set the state at time t from host arrays, copied: k[nmat][ny][nx] volume
 * fractions (>= 0, each cell sums to 1 within 1e-12), rho and e [nmat][ny][nx]
 * per-material density (> 0) and specific internal energy (>= 0) where k > 0
 * (ignored elsewhere), ux, uy [ny+1][nx+1] nodal velocities (the wall-normal
 * component on wall nodes is set to 0).  Partial volumes are k dx dy, masses
 * rho V, energies M e.  Computes the first CFL time step; synchronizes. */
int lr_set_state(lr_ctx *c, double t, const double *k, const double *rho,
                 const double *e, const double *ux, const double *uy);

/* As lr_set_state, from DEVICE arrays of the same shapes (dtype LR_F64:
 * double, LR_F32: float), copied on the context's stream.  The checks of
 * lr_set_state run on the device; synchronizes. */
enum { LR_F64 = 0, LR_F32 = 1 };
int lr_set_state_device(lr_ctx *c, double t, const void *k, const void *rho,
                        const void *e, const void *ux, const void *uy, int dtype);

/* One time step (Lagrangian phase, DirectCF remap with partial VOF fluxes,
 * momentum remap; paper §1.2, §2.3, §4.1, §4.4).  *dt_out (may be NULL)
 * receives the step used.  Synchronizes. */
int lr_step(lr_ctx *c, double *dt_out);

/* Step until t reaches t_end (the last step is shortened to land on it) or
 * max_steps steps were taken.  The time step is chosen on the device; the
 * host checks completion every few steps only.  *steps_out, *t_out may be
 * NULL.  Synchronizes. */
int lr_run(lr_ctx *c, double t_end, long max_steps, long *steps_out, double *t_out);

/* Copy the fields selected by field_mask into caller-allocated host arrays,
 * out[0..popcount(mask)-1] in increasing bit order (shapes above). */
int lr_get_fields(lr_ctx *c, unsigned field_mask, double *const *out);

/* FP64 totals, out[3*nmat+3]: sum V_a, sum M_a, sum E_a per material, then
 * sum w m_p u_x, sum w m_p u_y and the total energy sum E_a + sum w m_p |u|^2/2
 * (m_p = 1/4 of the adjacent cell masses, w = 1, 1/2 on walls, 1/4 at corners). */
int lr_totals(lr_ctx *c, double *out);

/* Copy a named intermediate array of the last step into out (host), for
 * stage-by-stage checks (all but "dt", "t", "eL", "mp", "uh*", "uL*", "dp*",
 * "muX", "muY", "muD", "muA" need opts.stages = 1): "dt", "t", "Q", "S",
 * "volcf", "VL" [ny][nx];
 * "eL", "rhocf", "P_half" [nmat][ny][nx]; "mp", "uhx", "uhy", "uLx", "uLy",
 * "dpx", "dpy", "muD", "muA" [ny+1][nx+1]; "muX" [ny][nx+1]; "muY" [ny+1][nx];
 * "Wpx" [nmat][ny][nx+1]; "Wpy" [nmat][ny+1][nx]; "Wpc" [nmat][ny+1][nx+1];
 * "dxL", "dyL" [ny][nx].  Fluxes are signed along +x, +y, the main diagonal
 * (SW->NE) or the anti-diagonal (NW->SE).  "run" [4] (no stages needed): the
 * capacity of the mixed-cell list, 1 if full chunks of lr_run replay a
 * captured HIP graph (0 before the first, or if capture failed), 1 if
 * capture failed, the tile shape of the step kernels (LR_TILE_*). */
int lr_debug_get(lr_ctx *c, const char *name, double *out);

/* Kernel timing for benchmarks.  lr_profile(c, 1) makes every later step
 * launch its kernels with a start/stop HIP event pair recorded by the
 * dispatch itself on the context's stream (kernel execution time only);
 * lr_profile_read adds up the elapsed milliseconds and the
 * launch counts per kernel into ms[n], counts[n] (n <= lr_kernel_count(), in
 * the order of lr_kernel_name(i)) and resets them.  Off by default. */
int lr_profile(lr_ctx *c, int enable);
int lr_profile_read(lr_ctx *c, double *ms, long *counts, int n);
int lr_kernel_count(void);
const char *lr_kernel_name(int i);

/* ------------------------------------------------------------------ batch
 * Many independent problems of different grid sizes stepped together: each
 * kernel of a step is one launch over the tiles of every running problem of
 * the batch, optionally replayed from a HIP graph.  Problems
 * are admitted while others run (continuous batching): a submitted problem
 * takes a free slot and a range of the batch's device pool, starts with the
 * next chunk of steps and leaves the launches when it finishes; its state
 * stays resident until released.  Every problem of a batch has the batch's
 * nmat and precision.  Each problem's arithmetic is that of a single context
 * (its own time step, same kernels), so its result is the same alone and in
 * any mix.  One host thread at a time per batch. */
typedef struct {
  int max_slots;        /* problems resident at once (>= 1)                      */
  size_t pool_bytes;    /* device memory for problem state, allocated at create  */
  int nmat;             /* materials of every problem                            */
  int precision;        /* LR_FP64 or LR_FP32                                     */
  int chunk_steps;      /* steps per lr_batch_step (even, >= 2); default 16      */
  int use_graph;        /* 1: replay each chunk from a captured HIP graph        */
  int persistent;       /* 1: grids limited to the blocks resident on the device, each
                           block walking the tile list; 0 (default): one block per tile */
  int autotune;         /* 1: the first chunks time every schedule (persistent x
                           use_graph x tile, LR_NSCHED of them) on the device, in
                           one order and then the reverse (a drift of the cost as
                           the flow develops cancels to first order); the fastest
                           per cell-step is kept (persistent, use_graph and tile
                           are then ignored).  Results do not depend on it. */
  int tile;             /* tile shape of the step kernels: LR_TILE_32x8 (default),
                           LR_TILE_16x16, LR_TILE_32x16 or LR_TILE_32x12 (cells per
                           block in x by y; 32x16 blocks have 512 threads, 32x12
                           384).  Results do not depend on it. */
} lr_batch_opts;
enum { LR_TILE_AUTO = -1, LR_TILE_32x8 = 0, LR_TILE_16x16 = 1, LR_TILE_32x16 = 2, LR_TILE_32x12 = 3 };
#define LR_NTILE 4
/* schedules the autotuner times: c = persistent + 2*use_graph + 4*tile, over
 * the first LR_NTUNE_TILE shapes (32x12 is the shape of small single grids) */
#define LR_NTUNE_TILE 3
#define LR_NSCHED (4 * LR_NTUNE_TILE)
typedef struct lr_batch lr_batch;

void lr_batch_default_opts(lr_batch_opts *o);
int lr_batch_create(const lr_batch_opts *o, lr_batch **out);
int lr_batch_bind_stream(lr_batch *b, void *hip_stream);
/* device bytes of the pool one problem of this size takes */
size_t lr_batch_footprint(int nx, int ny, int nmat, int precision);
/* Admit a problem: grid nx x ny, eos[nmat], opts as for lr_create (its
 * precision must be the batch's; stages must be 0; NULL = defaults), initial
 * state at t = 0 as for lr_set_state (host arrays, copied), run until t_end
 * or max_steps steps.  *req_id receives its id (>= 0).  LR_EAGAIN: no free
 * slot or no pool range large enough now (retry after a release). */
int lr_batch_submit(lr_batch *b, int nx, int ny, const lr_eos *eos, const lr_opts *opts,
                    double t_end, long max_steps, const double *k, const double *rho,
                    const double *e, const double *ux, const double *uy, long *req_id);
/* Run one chunk of opts.chunk_steps steps of every running problem, then
 * check which finished.  *n_running (may be NULL) receives the number still
 * running.  Synchronizes. */
int lr_batch_step(lr_batch *b, int *n_running);
/* lr_batch_step in two halves, so that host work (admissions of new
 * requests) runs while the chunk does: begin launches the chunk and returns
 * at once; end waits for it and then behaves as lr_batch_step's check.
 * Between the two, submit and release may be called, and poll, status,
 * get_fields and totals on requests that are not running (a request
 * submitted meanwhile joins at the next begin).  Begin while a chunk is in
 * flight is LR_EINVAL, and so is lr_batch_bind_stream; end with none in
 * flight only counts. */
int lr_batch_step_begin(lr_batch *b);
int lr_batch_step_end(lr_batch *b, int *n_running);
/* Ids of problems that finished (t_end or max_steps reached, or failed)
 * since the last poll, at most cap of them; *n receives the count. */
int lr_batch_poll(lr_batch *b, long *ids, int cap, int *n);
/* rc: LR_OK, a failure code of the problem, or LR_EAGAIN while it runs;
 * steps taken and time reached (any may be NULL). */
int lr_batch_status(lr_batch *b, long id, int *rc, long *steps, double *t);
/* as lr_get_fields / lr_totals for one resident problem */
int lr_batch_get_fields(lr_batch *b, long id, unsigned field_mask, double *const *out);
int lr_batch_totals(lr_batch *b, long id, double *out);
/* free the problem's slot and pool range */
int lr_batch_release(lr_batch *b, long id);
int lr_batch_running(lr_batch *b);
/* the schedule in use (any pointer may be NULL); rates[LR_NSCHED] receives
 * the cell-steps per ms the autotuner measured for schedules
 * c = persistent + 2*use_graph + 4*tile.  LR_EAGAIN while it is still timing. */
int lr_batch_schedule(lr_batch *b, int *persistent, int *use_graph, int *tile, double *rates);
const char *lr_batch_last_error(const lr_batch *b);
void lr_batch_destroy(lr_batch *b);

/* ------------------------------------------------------- allocation-free
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): lr_create,
 * lr_set_state_device (FP64 inputs), lr_run and the copy of lr_get_fields in
 * one call that allocates nothing.  Every device array of the problem (state,
 * intermediates, control record, block maps) is carved from a static
 * workspace of LR_NOALLOC_BYTES bytes, one per device, which the library
 * holds from the first call on that device until the process ends.  The
 * caller passes the inputs and outputs:
 *   nx, ny, nmat, eos, bc, opts: as lr_create (opts.stages must be 0);
 *   t0, t_end, max_steps: the state is at t0; the run stops at t_end or after
 *     max_steps steps, as lr_run;
 *   k, rho, e [nmat][ny][nx], ux, uy [ny+1][nx+1]: DEVICE FP64 arrays, the
 *     initial state with the checks of lr_set_state (run on the device);
 *   field_mask, out: out[0..popcount(mask)-1] are DEVICE FP64 arrays of the
 *     shapes of lr_get_fields, written in increasing bit order;
 *   hip_stream: the hipStream_t to run on (NULL: the null stream);
 *   steps_out, t_out (may be NULL): steps taken and time reached;
 *   errbuf[errlen] (may be NULL): the failure text.
 * A problem whose arrays do not fit in the workspace (about 265 bytes per
 * cell for FP64 with 3 materials, so up to about 240,000 cells) is LR_ENOMEM,
 * with the sizes in errbuf.  Every call on a device shares that device's
 * workspace, and the workspace keeps the last call's contents: calls that
 * overlap on one device (other host threads, other streams) race, so callers
 * serialize them.  Synchronizes the stream. */
#define LR_NOALLOC_BYTES ((size_t)64 << 20)
int lr_run_noalloc(int nx, int ny, int nmat, const lr_eos *eos, const int bc[4],
                   const lr_opts *opts, double t0, double t_end, long max_steps,
                   const double *k, const double *rho, const double *e,
                   const double *ux, const double *uy, unsigned field_mask,
                   double *const *out, void *hip_stream, long *steps_out,
                   double *t_out, char *errbuf, size_t errlen);

/* Text of the last failure on this context; valid until the next call. */
const char *lr_last_error(const lr_ctx *c);

/* Free the context and its device memory (NULL is ignored). */
void lr_destroy(lr_ctx *c);

#ifdef __cplusplus
}
#endif
#endif
