/*
 * lr_ref.h — oracle for the 2D multimaterial Lagrange–Remap step with the
 * one-step "Direct remap with Corner Fluxes" (DirectCF) of
 * B. Chaudet, "A scalable Lagrange-Remap scheme for compressible
 * multimaterial Euler equations with sharp interface reconstruction"
 * (arXiv:2208.13409).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is a plain, slow, FP64 CPU
 * implementation used to check the GPU library.  Only the test suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no source with the GPU library; it exports the same call shapes with
 * an lr_ref_ prefix so a test can drive both with the same inputs.
 *
 * All functions return 0 on success and a negative code on failure; they
 * never abort.  All arrays are host memory, FP64, row-major with x fastest.
 *
 * Pins: the physics and closed-form pins of the test suite, and a second
 * reader of the whole step in 50-digit arithmetic on tiny grids.  Four
 * readings where the paper is silent are fixed by no value the paper prints
 * (only both readers, conservation and bounds constrain them): the discrete
 * divergence inside the pseudo-viscosity, the dual-mesh reconstruction
 * geometry, the interface rule for cells with three or more materials, and
 * the way clipping hands a material's excess outflow to the donor's other
 * materials.
 */
#ifndef LR_REF_H
#define LR_REF_H
#ifdef __cplusplus
extern "C" {
#endif

#define LR_REF_MAXMAT 4
/* branch counters returned by lr_ref_debug_get(c, "counts", out[LR_REF_NCOUNT]):
 * cells, summed over the steps since set_state, that were mixed, had three or
 * more materials, had a degenerate Youngs normal, had a material's outflow
 * clipped, or fell back to order 1 under the positivity guard */
#define LR_REF_NCOUNT 5

/* equation of state of one material: p = (gamma - 1) rho e - pinf, the
 * perfect gas of §5.1 for pinf = 0 and the stiffened gas of §5.2 (the paper's
 * pi) for pinf > 0; gamma > 1, pinf >= 0 */
typedef struct { double gamma, pinf; } lr_ref_eos;

typedef struct {
  double x0, x1, y0, y1;  /* domain; dx = (x1-x0)/nx, dy = (y1-y0)/ny          */
  double cfl;             /* CFL number (default 0.5)                            */
  double a1, a2;          /* Wilkins linear / quadratic coefficients (0.5, 1.0)  */
  int precision;          /* ignored by the oracle: always FP64                  */
  int recon_order;        /* 1 = upwind everywhere, 2 = limited linear along each
                             direction (default), 3 = the multidimensional
                             least-squares plane of §3.3 (DirectCF only)         */
  int kinematic;          /* 1 = prescribed node velocities, no forces           */
  double k_eps;           /* material-presence threshold on V/A (default 1e-10)  */
  double fixed_dt;        /* > 0: use this time step instead of the CFL one      */
  int remap;              /* LR_REF_REMAP_DIRECTCF (default) or LR_REF_REMAP_AD  */
} lr_ref_opts;

/* remap of the time step: the one-step DirectCF remap (§2.3), or the
 * alternate-direction comparator (§2.1.1-§2.1.2, §4.2) */
enum { LR_REF_REMAP_DIRECTCF = 0, LR_REF_REMAP_AD = 1 };

enum { LR_REF_OK = 0, LR_REF_EINVAL = -1, LR_REF_ENOMEM = -2, LR_REF_EDEVICE = -3,
       LR_REF_ENEGATIVE = -4, LR_REF_ENAN = -5, LR_REF_EDT = -6, LR_REF_EAGAIN = -7,
       LR_REF_ESTATE = -8 };

/* field mask bits for lr_ref_get_fields; per-material fields are [nmat][ny][nx],
 * mixture fields [ny][nx], node fields [ny+1][nx+1] */
enum { LR_REF_F_RHO = 1, LR_REF_F_P = 2, LR_REF_F_E = 4, LR_REF_F_K = 8,
       LR_REF_F_RHOA = 16, LR_REF_F_EA = 32, LR_REF_F_PA = 64, LR_REF_F_UX = 128,
       LR_REF_F_UY = 256, LR_REF_F_VOL = 512, LR_REF_F_MASS = 1024, LR_REF_F_IE = 2048 };

typedef struct lr_ref_ctx lr_ref_ctx;

void lr_ref_default_opts(lr_ref_opts *o);
int lr_ref_create(int nx, int ny, int nmat, const lr_ref_eos *eos, const int bc[4],
                  const lr_ref_opts *opts, lr_ref_ctx **out);
int lr_ref_set_state(lr_ref_ctx *c, double t, const double *k, const double *rho,
                     const double *e, const double *ux, const double *uy);
int lr_ref_step(lr_ref_ctx *c, double *dt_out);
int lr_ref_run(lr_ref_ctx *c, double t_end, long max_steps, long *steps_out, double *t_out);
int lr_ref_get_fields(lr_ref_ctx *c, unsigned mask, double *const *out);
/* out[3*nmat+3]: sum V_a, sum M_a, sum E_a (per material), sum w m_p u_x,
 * sum w m_p u_y, total energy; w = 1 inside, 1/2 on walls, 1/4 at corners */
int lr_ref_totals(lr_ref_ctx *c, double *out);
/* stage arrays of the last step (names listed in lr_ref.c), and "counts" */
int lr_ref_debug_get(lr_ref_ctx *c, const char *name, double *out);
const char *lr_ref_last_error(const lr_ref_ctx *c);
void lr_ref_destroy(lr_ref_ctx *c);

/* geometry kernels exposed for the unit pins */
double lr_ref_rect_halfplane_area(double x0, double x1, double y0, double y1,
                                  double nx, double ny, double s);
double lr_ref_interface_offset(double x0, double x1, double y0, double y1,
                               double nx, double ny, double frac);

#ifdef __cplusplus
}
#endif
#endif
