/*
 * orc.h -- C interface of the CPU FP64 oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle is a plain, slow, obviously
 * correct CPU implementation of the patch-update method (guard fill by
 * linear time interpolation, quantised local time steps, MUSCL-Hancock +
 * HLLD + constrained transport, readiness-driven dispatcher).  Only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code with the GPU library: the two are written
 * independently and meet only through the seeded input generators.
 *
 * The calls mirror the GPU library's boundary with the prefix orc_.
 * Return codes: 0 ok, <0 error (same numbering as the GPU library).
 */
#ifndef ORC_H
#define ORC_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EKMAX = -4, ORC_EALIGN = -5,
       ORC_ENONFINITE = -6, ORC_ENEGATIVE = -7, ORC_ESTATE = -8 };

typedef struct {
  double gamma, courant, dt_base, dt_fixed, grace, p_floor;
  int32_t kmax, nslots, nguard, limiter;
  int32_t prec;    /* ignored: the oracle always computes in FP64 */
  int32_t dt_mode; /* 0 LOCAL, 1 GLOBAL_QUANT, 2 GLOBAL_EXACT, 3 FIXED */
  int32_t periodic[3];
  double box_lo[3], box_hi[3];
  /* non-ideal MHD (Sec. 4.3): Ohmic resistivity eta_Ohm, ambipolar drift
   * coefficient gamma_AD and ion density rho_i; 0, 0 = ideal */
  double eta, gamma_ad, rho_ion;
  /* order of the guard-zone time interpolation: 0 or 1 linear, 2 quadratic
   * through three slices (Sec. 3B) */
  int32_t torder;
} orc_config;

/* flags: bit 0 = boundary patch (never updated; its one slice is the value
 * at every time, and readiness ignores it; LOCAL mode only) */
typedef struct {
  double origin[3], size[3];
  int32_t n, level;
  int32_t flags;
} orc_patch_desc;

typedef struct orc_set orc_set;

int orc_create(const orc_config* cfg, const orc_patch_desc* pd, int32_t npatch, orc_set** out);
int orc_init(orc_set* s, const double* U, size_t n_values, double t0);
int orc_advance_to(orc_set* s, double t_end);
int orc_read_state(const orc_set* s, double* U, size_t n_values, double* t_out);
int orc_read_schedule(const orc_set* s, int64_t* steps, uint64_t* khash, int32_t* klog,
                      size_t klog_cap);
int orc_stats(const orc_set* s, double out[16]);
void orc_destroy(orc_set* s);
const char* orc_last_error(void);

/* Oracle-only controls and probes. */
/* order: 0 = oldest-first (ticks, id); 1 = uniformly random ready patch (seeded);
 * 2 = rounds: the whole ready set at once, updated by nthreads threads. */
int orc_set_order(orc_set* s, int32_t order, uint64_t seed, int32_t nthreads);
/* LOCAL mode: stop after max_updates patch updates (sequential orders) or
 * max_updates rounds (order 2). */
int orc_advance_limited(orc_set* s, double t_end, int64_t max_updates);
/* Current time of every patch (ticks and/or double). */
int orc_times(const orc_set* s, int64_t* ticks, double* t);
/* Number of values per patch slice and per-patch offsets (npatch+1 entries). */
int orc_layout(const orc_set* s, int64_t* offsets);
/* Number of updates whose guard fill extrapolated a neighbour in time (a
 * grace g > 0 let the patch run ahead of that neighbour). */
int orc_extrapolated(const orc_set* s, int64_t* count);
/* Symmetric neighbour lists: counts[npatch], then ids (capacity cap). */
int orc_nbors(const orc_set* s, int32_t* counts, int32_t* ids, size_t cap);
/* Guard-filled padded array of patch p at its current time: layout of the
 * padded patch (5 cell arrays of N^3, N = n + 2*nguard, then Bx, By, Bz). */
int orc_padded(const orc_set* s, int32_t p, double* out, size_t n_values);
/* Slice rel = 0 (latest), 1 (previous), ... of patch q with its time. */
int orc_slot(const orc_set* s, int32_t q, int32_t rel, double* out, size_t n_values,
             int64_t* ticks, double* t);
/* Single HLLD interface flux: w = (rho, un, ut1, ut2, p, bt1, bt2); flux8 =
 * (mass, mn, mt1, mt2, energy, bt1, bt2, upwind speed). */
int orc_hlld_flux(const double* wl, const double* wr, double bn, double gamma, double eps,
                  double* flux8);
/* Forward-mode derivative (exact JVP along the taken branches) of nsteps
 * FIXED steps of the whole set: U0 + eps*dU0 -> UT + eps*dUT. */
int orc_jvp_fixed(orc_set* s, const double* U0, const double* dU0, int32_t nsteps, double dt,
                  double* UT, double* dUT);

/* Arithmetic work of the method: floating-point operations (+, -, *, /,
 * sqrt, one each) and cell updates from state U0 (slice layout) to t_end,
 * same configuration, one thread.  out[0] = operations, out[1] = updates,
 * out[2] = the operations of the Courant rate (included in out[0]). */
int orc_count_flops(orc_set* s, const double* U0, double t_end, double* out);

#ifdef __cplusplus
}
#endif
#endif
