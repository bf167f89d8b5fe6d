/* dycore.h - C ABI of the MI355X leap-format dynamical-core step.
 *
 * The library advances the four forecast variables of the IAP-transformed
 * primitive equations (eq. 1 of AGCM-3DLF, arXiv 2103.10114): zonal wind U,
 * meridional wind V, temperature variable Phi and surface pressure p_s, on the
 * latitude-longitude-sigma Arakawa C grid (Sec. III-B).  Zonal differences use
 * the leap format (eq. 6) with the per-latitude span of eq. 7 and the leap
 * patterns of Table VII; a step is the split of eq. 2 with 3M adaptation and 3
 * advection calls (Sec. III-D, message aggregation).
 *
 * Layout of every field: contiguous [j][k][i], longitude i fastest, then
 * level k (top to surface), then latitude row j from the north pole.
 *   U   : (ny+1) x nz x nx  at (i+1/2, j); pole rows are ignored on input and written 0
 *   V   :  ny    x nz x nx  at (i, j+1/2), positive toward increasing colatitude
 *   Phi : (ny+1) x nz x nx  at (i, j); each pole row holds one value (read as the row mean)
 *   p_s : (ny+1) x nx       at (i, j), Pa; pole rows as Phi
 * Every field pointer is a device pointer to float (DYCORE_FP32) or double
 * (DYCORE_FP64), aligned to 16 bytes.  The caller owns all field buffers.
 *
 * Streams: `stream` is a hipStream_t passed as void*; NULL is the default
 * stream.  step / stage / adjoint calls only enqueue work, allocate nothing
 * and never synchronise the host.  A handle is not thread safe.
 *
 * Errors: every call returns a dycore_status.  Argument errors are reported
 * synchronously and enqueue nothing.
 */
#ifndef DYCORE_H
#define DYCORE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dycore_s* dycore_t;

typedef enum {
  DYCORE_OK = 0,
  DYCORE_EINVAL = -1,       /* bad argument: NULL, size, alignment, dt, ... */
  DYCORE_ENOMEM = -2,       /* device allocation failed in create */
  DYCORE_EHIP = -3,         /* a HIP runtime call or kernel launch failed */
  DYCORE_ENONFINITE = -4,   /* a field holds NaN or Inf (dycore_check_finite) */
  DYCORE_EUNSUPPORTED = -5  /* grid too large for a kernel's tile limits */
} dycore_status;

typedef enum { DYCORE_FP32 = 0, DYCORE_FP64 = 1 } dycore_precision;

enum {
  DYCORE_FORWARD_ONLY = 1u,   /* do not reserve adjoint workspace at create */
  DYCORE_LOWLAT_FILTERS = 2u, /* close every outer step with the low-latitude filters the leap format
                                 keeps (Sec. III-B, Table IV rows 1-2): below 38 degrees the
                                 simplified filter removes the 2-dlam wave of each zonal row, from 38
                                 to 70 degrees the 3-point operator F + r (F_{x-1} - 2F + F_{x+1})
                                 with r = (1 - cos(lat)/cos 38deg)/4; on U, V, Phi and p_s, pole rows
                                 untouched.  Needs an even nx (EINVAL otherwise). */
  DYCORE_SINGLE_STREAM = 4u   /* run every launch on the caller's stream: no second stream, so the
                                 advection's polar tiles and the stage adjoints' pole-row chains run
                                 before and after the other tiles instead of beside them.  Results are
                                 bitwise the same; only the schedule differs. */
};

typedef struct {
  int nx;                  /* longitudes, >= 8, <= 4096 */
  int ny;                  /* latitude intervals (ny+1 scalar rows incl. both poles), >= 4 */
  int nz;                  /* sigma levels, >= 1, <= 128; nx (ny+1) (nz+1) x element size < 4 GiB */
  double dt;               /* outer time step, seconds, > 0 */
  int n_adapt_substeps;    /* M of Sec. III-D; 0 = from the CFL bound ceil(w_max dt / (0.8 sqrt 3));
                              a given M below that bound (dt / M above the CFL limit) is EINVAL */
  int prec;                /* dycore_precision of every field pointer */
  const double* sigma_half;/* host, nz+1 increasing values from 0 to 1, or NULL for uniform */
  const double* phis;      /* host, (ny+1)*nx surface geopotential (m^2/s^2), copied; NULL = flat */
  double a, omega, g, rd, cp, p0, t0;  /* constants; 0 selects 6.371e6, 7.292e-5, 9.80616,
                                          287.04, 1004.64, 1e5, 300 */
  unsigned flags;          /* DYCORE_FORWARD_ONLY | DYCORE_LOWLAT_FILTERS | DYCORE_SINGLE_STREAM */
  int block;               /* threads per workgroup of the tiled advection stage (64..1024, multiple of
                              64; sizes above 256 run as 256); 0 = 256.  Results do not depend on it. */
  double kappa_star;       /* kappa* of eq. 1's p_s line (m^2/s, >= 0; 0 = off): the adaptation's p_s
                              tendency gains kappa* D_sa, D_sa the flux-form horizontal Laplacian of
                              p_s (leaped second difference zonally, cap fluxes at the poles) */
} dycore_config;

/* Create a handle: validates the config, builds the leap table (eq. 7; span made
 * odd, Sec. III-B) and geometry, uploads them and reserves all scratch.
 * Returns DYCORE_EINVAL (bad config), DYCORE_ENOMEM, DYCORE_EHIP. */
int dycore_create(const dycore_config* cfg, dycore_t* out);

/* Release the handle and everything it owns.  Waits for its device work. */
int dycore_destroy(dycore_t h);

/* Advance (U, V, Phi, p_s) in place by nsteps outer steps (eq. 2 split:
 * M RK3 sub-steps of the adaptation with dt/M, then one RK3 step of the
 * advection with dt).  nsteps >= 0. */
int dycore_step(dycore_t h, void* U, void* V, void* Phi, void* ps, int nsteps, void* stream);

/* n_rk RK3 steps of one process alone (0 adaptation, 1 advection) with step
 * hstep, in place: the 3 stage launches per RK step are those of dycore_step.
 * Used to integrate or time one process of the split on its own. */
int dycore_process_run(dycore_t h, int process, int n_rk, double hstep, void* U, void* V, void* Phi, void* ps,
                       void* stream);

/* One stage: out = base + ch * T(in), T the adaptation (process 0) or advection
 * (process 1) tendency of eq. 2; pole rows of out hold the base row mean plus
 * ch times the pole tendency, U pole rows 0.  out may alias base (not in). */
int dycore_stage(dycore_t h, int process, double ch,
                 const void* bU, const void* bV, const void* bPhi, const void* bps,
                 const void* U, const void* V, const void* Phi, const void* ps,
                 void* oU, void* oV, void* oPhi, void* ops, void* stream);

/* Adjoint of one outer step about its start state (U0, V0, Phi0, ps0), under
 * the Euclidean inner product over every stored entry.  On entry (aU, aV,
 * aPhi, aps) hold the adjoint of the step's output; on return, the adjoint of
 * its input.  Recomputes the forward stages internally.  Needs the adjoint
 * workspace (a handle created without DYCORE_FORWARD_ONLY). */
int dycore_step_adjoint(dycore_t h, const void* U0, const void* V0, const void* Phi0, const void* ps0,
                        void* aU, void* aV, void* aPhi, void* aps, void* stream);

/* One outer step in place, as dycore_step with nsteps = 1 (same kernels, same result bit for bit),
 * that also keeps the step's 3(M+1) stage inputs in the handle's adjoint workspace, so that
 * dycore_step_adjoint_recorded can sweep back without recomputing them (storing instead of
 * recomputing the forward stages of one step, as an adjoint of a just-taken step needs).  Needs
 * the adjoint workspace: DYCORE_EINVAL for a DYCORE_FORWARD_ONLY handle or NULL fields. */
int dycore_step_record(dycore_t h, void* U, void* V, void* Phi, void* ps, void* stream);

/* Adjoint of the step last taken with dycore_step_record, equal to dycore_step_adjoint about that
 * step's start state: (aU..aps) hold the adjoint of the step's output on entry and of its input
 * on return.  The recorded stages stay valid for further calls (other adjoint seeds) until the
 * next dycore_step_record or dycore_step_adjoint on the handle; DYCORE_EINVAL when none is held. */
int dycore_step_adjoint_recorded(dycore_t h, void* aU, void* aV, void* aPhi, void* aps, void* stream);

/* Adjoint of one stage about its input (U..ps): adds J_base^T a_out into
 * (abU..) and J_in^T a_out into (aiU..).  The two accumulators may be the
 * same buffers (the stage's base and input then coincide); neither may alias
 * a_out.  Needs the adjoint workspace. */
int dycore_stage_adjoint(dycore_t h, int process, double ch,
                         const void* U, const void* V, const void* Phi, const void* ps,
                         const void* aoU, const void* aoV, const void* aoPhi, const void* aops,
                         void* abU, void* abV, void* abPhi, void* abps,
                         void* aiU, void* aiV, void* aiPhi, void* aips, void* stream);

/* FP64 global mass (sum_j w_j sum_i p_s + cap areas times the pole values) and the quadratic
 * energy measure (p0/2g) sum w dsig (U^2 + V^2 + Phi^2) + (R T0 p0/2g) sum w q^2: the conserved
 * quantities whose drift Sec. IV-B follows.  Both sums run on the device in a fixed order (row
 * partials, then one fixed-order reduction); only the two scalars are copied to the host doubles
 * (synchronises the stream).  EINVAL on NULL arguments. */
int dycore_diagnostics(dycore_t h, const void* U, const void* V, const void* Phi, const void* ps,
                       double* mass_out, double* energy_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops
 * that forbid hipMalloc): dycore_diagnostics with its row partials in a static device array of the
 * library (3 (ny+1) doubles, at most 4097 rows, one copy per GPU held until the process ends) and
 * the results written to device memory, out_dev[0] = mass and out_dev[1] = energy, without copying
 * to the host or synchronising.  Allocates nothing.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other threads) race.  Results equal
 * dycore_diagnostics bit for bit.  EINVAL: NULL arguments or ny + 1 > 4097. */
int dycore_diagnostics_noalloc(dycore_t h, const void* U, const void* V, const void* Phi, const void* ps,
                               double* out_dev, void* stream);

/* Count of non-finite stored entries in the four fields (synchronises the
 * stream).  Returns DYCORE_ENONFINITE if the count is positive. */
int dycore_check_finite(dycore_t h, const void* U, const void* V, const void* Phi, const void* ps,
                        long long* count_out, void* stream);

/* Leap spans (odd, eq. 7): ny+1 values for scalar/U rows (1 at the poles) and ny for V rows. */
int dycore_leap_table(dycore_t h, int* m_rows, int* m_vrows);

/* Adaptation sub-steps M in use; block size in use. */
int dycore_substeps(dycore_t h);
int dycore_block(dycore_t h);

/* Bytes of device memory the handle holds. */
size_t dycore_workspace_bytes(dycore_t h);

/* Live timing of the row-fused adaptation-stage adjoint kernel (the dominant kernel of
 * dycore_step_adjoint and dycore_step_adjoint_recorded; Sec. III-D, eq. 6, transposed):
 * start makes 2 max_launches HIP events (host call, allocates; not for a timed region) and
 * arms the handle; every later launch of that kernel on the handle, up to max_launches, is
 * bracketed by events recorded on its launch stream.  stop waits for the last recorded event,
 * writes the sum of the bracketed durations (ms) and the number of timed launches, disarms
 * and frees the events.  DYCORE_EINVAL: NULL arguments, max_launches outside 1..65536, stop
 * without start; DYCORE_EHIP: event creation or query failed (the timer is released). */
int dycore_kernel_timer_start(dycore_t h, int max_launches);
int dycore_kernel_timer_stop(dycore_t h, double* total_ms, int* launches);

/* Batches of ensemble members (any grids, one precision) advanced together:
 * one persistent launch per global stage, each workgroup pulling (member,
 * zonal tile) work items, so the launch sequence of a step is fixed and can be
 * captured once in a hipGraph and replayed.
 *
 * dycore_batch_create binds member m's fields (U[m], V[m], Phi[m], ps[m],
 * device pointers of its handle's grid) and uploads the stage descriptors; it
 * allocates and synchronises.  Each member needs its own handle (the handle's
 * scratch is used).  block = threads per workgroup (0: 256; above 512:
 * DYCORE_EUNSUPPORTED), grid = persistent workgroups (0: fill every CU).
 * dycore_batch_step only enqueues kernels and gives results equal bit for bit
 * to dycore_step on each member. */
typedef struct dycore_batch_s* dycore_batch_t;
int dycore_batch_create(int n, const dycore_t* hs, void* const* U, void* const* V, void* const* Phi,
                        void* const* ps, int block, int grid, dycore_batch_t* out);
int dycore_batch_step(dycore_batch_t b, int nsteps, void* stream);
int dycore_batch_destroy(dycore_batch_t b);

const char* dycore_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* DYCORE_H */
