/*
 * dsp.h -- C ABI of libdsp.so, the MI355X patch engine for ideal MHD with
 * local time steps (the DISPATCH method: Nordlund et al. 2018, MNRAS).
 *
 * A patch set is the paper's task list of patch tasks (Sec. 2.1-2.2): each
 * patch is a cube of n^3 cells whose state is kept as a ring of time slices
 * (Sec. 3A).  Advancing the set to a time repeatedly updates every patch that
 * is ready in the sense of Eq. (1) (Sec. 3B), until every patch has reached
 * that time (the task list "execute" of Sec. 2.2).  One patch update
 *   1. fills the patch's guard zones from its neighbours, interpolating
 *      linearly in time between the two stored slices that bracket the
 *      patch time (extrapolating from the two newest when a grace g > 0 let
 *      the patch run ahead), and in space (conservative prolongation /
 *      restriction) where the neighbour has another resolution (Sec. 3A);
 *   2. takes one second-order MUSCL-Hancock step with HLLD fluxes and
 *      constrained transport of face-centred B (Sec. 4.1, 4.3), with its own
 *      Courant time step quantised to dt_base * 2^-k (local time steps,
 *      Sec. 1, Sec. 5.2);
 *   3. publishes the new slice over the oldest one (Sec. 3A).
 * All of it runs in HIP kernels on the GPU; the host only validates
 * arguments, builds the static neighbour tables and launches.
 *
 * Conventions for every call:
 *  - returns 0 (DSP_OK) or a negative DSP_E* code; nothing is thrown across
 *    the ABI; dsp_last_error() gives a message for the calling thread;
 *  - "host" pointers are ordinary CPU memory owned by the caller; "device"
 *    pointers are GPU memory owned by the caller;
 *  - a set owns all the device memory it allocates and frees it in
 *    dsp_destroy(); a set is not thread-safe, distinct sets are independent.
 *
 * Host layout of a state (dsp_init, dsp_read_state): patches in id order,
 * per patch rho, mx, my, mz, E each [n][n][n] (z, y, x; x fastest), then
 * Bx [n][n][n+1], By [n][n+1][n], Bz [n+1][n][n]; every patch stores both of
 * its boundary faces.  Values per patch: 5 n^3 + 3 n^2 (n+1).  Always FP64
 * on the host; FP32 sets round on upload.  Units: mu0 = 1, so the magnetic
 * pressure is |B|^2 / 2.
 */
#ifndef DSP_H
#define DSP_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
  DSP_OK = 0,
  DSP_EINVAL = -1,      /* invalid argument or configuration */
  DSP_ENOMEM = -2,      /* device allocation failed */
  DSP_EHIP = -3,        /* a HIP runtime call failed */
  DSP_EKMAX = -4,       /* a patch needs a time-step level k > kmax */
  DSP_EALIGN = -5,      /* time not a multiple of dt_base (LOCAL / GLOBAL_QUANT) */
  DSP_ENONFINITE = -6,  /* non-finite state or signal speed */
  DSP_ENEGATIVE = -7,   /* non-positive density, or pressure without a floor */
  DSP_ESTATE = -8       /* call not valid in the set's current state */
};

typedef enum { DSP_F32 = 1, DSP_F64 = 2 } dsp_prec;

/* How time steps are chosen (Sec. 1, Sec. 5.2):
 *  LOCAL        each patch its own level k (dt = dt_base 2^-k), Eq. (1) dispatch
 *  GLOBAL_QUANT every patch takes the smallest quantised step of the set
 *  GLOBAL_EXACT every patch takes courant / max Courant rate (last step clipped)
 *  FIXED        every patch takes dt_fixed (last step clipped) */
typedef enum {
  DSP_DT_LOCAL = 0,
  DSP_DT_GLOBAL_QUANT = 1,
  DSP_DT_GLOBAL_EXACT = 2,
  DSP_DT_FIXED = 3
} dsp_dt_mode;

typedef struct {
  double gamma;    /* ratio of specific heats, > 1 */
  double courant;  /* Courant number C of the rate sum_d (|v_d| + c_f,d)/dx */
  double dt_base;  /* coarsest quantised step (LOCAL, GLOBAL_QUANT) */
  double dt_fixed; /* step of the FIXED mode */
  double grace;    /* g of Eq. (1), 0 <= g < 1; g > 0 needs LOCAL and nslots >= 3.
                    * A patch p is ready when t_p <= t_q + floor(g dt_q) (ticks)
                    * for every neighbour q, dt_q the step q took last (0 before
                    * its first), and no neighbour still needs p's oldest slice
                    * (the next slice is not newer than any neighbour) */
  double p_floor;  /* 0: non-positive pressure is DSP_ENEGATIVE; > 0: floor (counted) */
  int32_t kmax;    /* finest level, 0..40; times are integer ticks dt_base 2^-kmax */
  int32_t nslots;  /* time slices kept per patch, >= 2 (3 recommended) */
  int32_t nguard;  /* guard layers of the patch model, 2 or 3; the stencil reads 2 */
  int32_t limiter; /* 0 = van Leer (the only one) */
  dsp_prec prec;   /* stencil precision; times, weights and sums stay FP64 */
  dsp_dt_mode dt_mode;
  int32_t periodic[3]; /* must be 1, 1, 1 */
  double box_lo[3], box_hi[3];
  /* Non-ideal MHD (Sec. 4.3), all >= 0; eta = gamma_ad = 0 is ideal MHD.
   * eta: Ohmic resistivity, E += eta J (Eq. Ohm); gamma_ad > 0: ambipolar
   * diffusion, E += -v_D x B with v_D = J x B / (gamma_ad rho rho_ion)
   * (Eq. AD), rho_ion > 0.  J = curl B on the edges of constrained transport,
   * from the state at the start of the step; the energy flux carries the
   * Poynting flux of this field, so the removed magnetic energy becomes heat
   * J.E.  The step also obeys dt <= 0.1 dx^2 / eta (Eq. dtOhm) and
   * dt <= 0.1 gamma_ad rho_ion rho dx^2 / B^2 (Eq. dtAD) in LOCAL and GLOBAL
   * modes.  Runs on the staged kernels; no adjoint. */
  double eta, gamma_ad, rho_ion;
  /* Order of the guard time interpolation (Sec. 3B): 0 or 1 linear between
   * the two bracketing slices; 2 quadratic through three slices (the pair and
   * the next older slice, else the next newer), Lagrange weights; needs
   * nslots >= 3, and a patch then also keeps the slice before any
   * neighbour's time.  Exact slice times are still plain copies. */
  int32_t torder;
} dsp_config;

/* One cubic patch: origin, edge length (size[0] == size[1] == size[2]),
 * interior cells n per edge (n >= 4), refinement level (informational).
 * Origins and sizes must lie on a common lattice: n/size integral and every
 * origin a multiple of 1/(2 lcm(n/size)).
 * flags: DSP_PATCH_FROZEN marks a boundary patch (the boundary tasks of
 * Sec. 3C, as a fixed state): it is never updated, its one slice is the
 * guard value at every time, and readiness ignores it.  LOCAL mode only;
 * at least one patch must be updated. */
enum { DSP_PATCH_FROZEN = 1 };
typedef struct {
  double origin[3], size[3];
  int32_t n, level;
  int32_t flags;
} dsp_patch_desc;

/* Optional device allocator (e.g. a framework's caching allocator).
 * NULL in dsp_create means hipMalloc / hipFree. */
typedef struct {
  void* ctx;
  void* (*alloc)(void* ctx, size_t bytes);
  void (*free)(void* ctx, void* p);
} dsp_allocator;

typedef struct dsp_set dsp_set;

/* Create a set of npatch patches (host arrays, copied).  Builds the
 * neighbour tables (symmetric closure of "reads guard data from", Eq. (1))
 * and allocates the time slices and work memory on the current device.
 * hip_stream: a hipStream_t to run on, or NULL for the default stream.
 * Errors: DSP_EINVAL (bad configuration or geometry), DSP_ENOMEM, DSP_EHIP. */
int dsp_create(const dsp_config* cfg, const dsp_patch_desc* patches, int32_t npatch,
               void* hip_stream, const dsp_allocator* alloc, dsp_set** out);

/* Upload a full state (host, FP64, n_values = total values of the layout
 * above) as the only valid slice of every patch, at time t0 (a multiple of
 * dt_base in LOCAL / GLOBAL_QUANT: restart).  Resets schedule and counters.
 * Errors: DSP_EINVAL (size), DSP_ENONFINITE, DSP_EALIGN, DSP_EHIP. */
int dsp_init(dsp_set* set, const double* U_host, size_t n_values, double t0);

/* Same as dsp_init, from a device array (host layout, in the set's precision,
 * caller-owned): a device-to-device copy, for re-running from a resident
 * initial state.  Errors: DSP_EINVAL, DSP_EALIGN, DSP_EHIP (no finiteness check). */
int dsp_init_device(dsp_set* set, const void* U_dev, double t0);

/* Advance every patch to t_end (Sec. 2.2 "execute").  Stream-ordered; returns
 * after completion.  Errors: DSP_EALIGN, DSP_EKMAX, DSP_ENONFINITE,
 * DSP_ENEGATIVE, DSP_EHIP; on error each patch is left at its last completed
 * step (dsp_read_state then returns those slices). */
int dsp_advance_to(dsp_set* set, double t_end);

/* Same as dsp_advance_to, but as the plain baseline: a host loop picks the
 * oldest ready patch (Sec. 3B mode (i)) and launches its update alone, one
 * patch per launch sequence, with a host round trip per update. */
int dsp_advance_to_plain(dsp_set* set, double t_end);

/* Download the latest slice of every patch (host, FP64, n_values as in
 * dsp_init).  t_out (nullable) receives the earliest patch time. */
int dsp_read_state(const dsp_set* set, double* U_host, size_t n_values, double* t_out);

/* Schedule record since dsp_init (host arrays of npatch entries): number of
 * updates per patch and an FNV-1a hash of its sequence of levels k (one byte
 * per update, k & 0xff, -1 in GLOBAL_EXACT / FIXED).  klog (nullable) receives
 * the first klog_cap levels per patch ([npatch][klog_cap], -2 past the end). */
int dsp_read_schedule(const dsp_set* set, int64_t* steps, uint64_t* khash, int32_t* klog,
                      size_t klog_cap);

/* Counters and FP64 diagnostics of the current state:
 *  [0] cell updates since init  [1] sum rho dV   [2..4] sum m dV   [5] sum E dV
 *  [6..8] sum B dV (cell means of faces)  [9] max |div B| (per unit length)
 *  [10] pressure-floor hits  [11] first-order fallback faces
 *  [12] GPU time of the last advance (ms)  [13] rounds (launch sequences)
 *  [14] earliest patch time  [15] latest patch time */
int dsp_stats(const dsp_set* set, double out[16]);

/* Time (ms, HIP events on the set's stream) of the dominant stencil kernel
 * summed over the last advance, and the number of its launches. */
int dsp_kernel_time(const dsp_set* set, double* ms, int64_t* launches);

/* Dominant-kernel record of the last advance (or fixed-step run):
 *  [0] GPU time (ms, HIP events on the set's stream) summed over the update
 *      launch sequences of the rounds: the fused step kernel, preceded by
 *      the cross-resolution guard resampling and the separate Courant pass
 *      when a round needs them
 *  [1] number of those launch sequences
 *  [2] their algorithmic HBM bytes: per patch update the own slice read and
 *      written plus every value of the two guard layers the stencil reads
 *      (all five cell variables of a guard cell, one component of a guard
 *      face), from one time slice (exact time) or two (interpolated)
 *  [3] 0: staged kernels (no byte count); 1: fused step kernel; 2: fused step
 *      kernel that also computed each patch's Courant rate and level (local
 *      steps of single-tile patches) */
int dsp_kernel_stats(const dsp_set* set, double out[4]);

/* Fixed-dt forward run for differentiation (all patches step together with
 * dt_fixed, nsteps steps).  U0_dev, UT_dev: device arrays in the host layout
 * and the set's precision (caller-owned).  ckpt_dev (nullable): device array of
 * (nsteps/8 + 1) states receiving the state every 8 steps (checkpointing). */
int dsp_fixed_steps_fwd(dsp_set* set, const void* U0_dev, void* UT_dev, int32_t nsteps,
                        void* ckpt_dev);

/* Reverse (adjoint) of nsteps fixed-dt steps: given lamT_dev = dJ/dU_T
 * (device, host layout, set precision), writes lam0_dev = dJ/dU_0, recomputing
 * forward states from the checkpoints written by dsp_fixed_steps_fwd.
 * seg: steps per checkpoint segment (must be 8).  The library allocates the
 * work buffers on first use: the forward intermediates of all 8 steps of a
 * segment when they take at most 16 GiB (each step is then recomputed once),
 * else of one step (each step recomputed twice). */
int dsp_fixed_steps_adj(dsp_set* set, const void* ckpt_dev, const void* lamT_dev,
                        void* lam0_dev, int32_t nsteps, int32_t seg);

/* Dispatch of LOCAL steps (Sec. 3B).  DSP_DISPATCH_ROUNDS: every round
 * updates the whole ready set (readiness scan, guard resampling, step,
 * publish as a queued launch sequence per round).  DSP_DISPATCH_QUEUE: the
 * paper's dispatcher mode (i) on the device -- one persistent kernel whose
 * workgroups take ready patches from a device queue, update and publish
 * them and push the neighbours that became ready, launched as a captured
 * hipGraph (queue seed + persistent kernel) replayed by each advance.  The
 * queue mode is available for single-precision sets without a grace whose
 * resampled guard boxes fit the staged resampling; a workgroup updates the
 * tiles of a larger patch (more than 16 cells per edge) one after another.
 * With g = 0 both modes give bitwise the same results.  New sets of patches
 * of at most 16^3 cells start in the queue mode when it is available, others
 * in the rounds (environment DSP_DISPATCH=rounds overrides).  Every wait of
 * the persistent kernel is bounded (DSP_QUEUE_TIMEOUT_S, default 30 s; then
 * DSP_ESTATE). */
enum { DSP_DISPATCH_ROUNDS = 0, DSP_DISPATCH_QUEUE = 1 };
/* Select the dispatch mode (DSP_EINVAL: the queue mode is not available for
 * this set) and, for the queue mode, the number of persistent workgroups
 * (0: one per compute unit, at most the number of patches). */
int dsp_set_dispatch(dsp_set* set, int32_t mode, int32_t workers);
/* Current mode, whether the queue mode is available, and its workgroups. */
int dsp_get_dispatch(const dsp_set* set, int32_t* mode, int32_t* queue_available, int32_t* workers);

/* Output cadence (Sec. 3E: each task writes its output when its time passes
 * its next output time, then advances that time by the interval).  From this
 * call on, every patch update whose new time t is a multiple of out_dt copies
 * the patch's new slice into frame (t / out_dt - 1) mod nframes of frames_dev:
 * a device array (current device, caller-owned, kept alive while the cadence
 * is set) of nframes frames, each the whole set in the host layout and the
 * set's precision (total values as for dsp_read_state).  Each patch writes its
 * own part of a frame when it reaches that time, independently of the others
 * (there is no barrier).  out_dt must be a positive multiple of dt_base: with
 * quantised steps every patch then reaches each output time exactly.  Needs
 * the LOCAL or GLOBAL_QUANT mode (DSP_EINVAL otherwise).  frames_dev null or
 * nframes <= 0 turns the cadence off. */
int dsp_set_output(dsp_set* set, double out_dt, void* frames_dev, int32_t nframes);
/* Autotuner: times LOCAL advances of t_probe (a multiple of dt_base) from the
 * set's current state with each candidate dispatch (rounds; the queue with
 * all, three quarters and half of the workgroups, when available), restores
 * the state, and selects the fastest.  cache_path (nullable): a text file of
 * JSON lines, one per tuned (device, set shape) key; an entry for this key
 * is used without timing, a new result is appended.  Allocates a copy of
 * the set's state for the duration of the call.  ms_out (nullable, 4
 * entries) receives the timings (-1: not a candidate). */
int dsp_autotune(dsp_set* set, double t_probe, const char* cache_path, double* ms_out);

/* Snapshot files (restart; output of the task list, Sec. 3E).  The file
 * holds the whole state of the set: for every patch (id order) its size and
 * level, time (ticks and FP64), current slot, step count, level hash and level
 * log, and every ring slot with its time, validity flag and values (host
 * layout, the set's precision).  Little-endian binary: the magic "DSPSNAP1",
 * int32 npatch, nslots, prec, kmax, log capacity, double dt_base, then the
 * per-patch records.  A set restored with dsp_load_snapshot (created with the
 * same patches and configuration) continues exactly as the saved one would
 * have.  Errors: DSP_EINVAL for file errors or a mismatching set, DSP_ESTATE
 * when saving an uninitialised set.  The caller owns the path. */
int dsp_save_snapshot(const dsp_set* set, const char* path);
int dsp_load_snapshot(dsp_set* set, const char* path);

/* HLLD flux (Miyoshi & Kusano 2005; the face flux of the step, Sec. 4.1) of
 * nface independent faces, evaluated on the current device with the step
 * kernels' own arithmetic in precision prec (DSP_F32: the hardware
 * reciprocal and square root of the single-precision step; DSP_F64: IEEE).
 * Host arrays, FP64, caller-owned: wl, wr [nface][7] rotated primitive
 * states (rho, u_n, u_t1, u_t2, p, B_t1, B_t2) left and right of the face
 * (rounded to prec on the device), bn [nface] the normal field; flux8
 * [nface][8] receives the fluxes of (rho, m_n, m_t1, m_t2, E, B_t1, B_t2) and
 * the upwind speed that orients the edge EMFs (S_L if S_L > 0, S_R if
 * S_R < 0, else the contact speed).  Independent of any set; allocates and
 * frees its own device buffers.  Errors: DSP_EINVAL, DSP_EHIP. */
int dsp_hlld_faces(int32_t prec, const double* wl, const double* wr, const double* bn, int64_t nface,
                   double gamma, double* flux8);

/* dsp_hlld_faces for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernel and arguments, but the device staging of the inputs and
 * outputs is a fixed file-scope device array of 12 MiB per GPU (held until
 * the process ends), so the call makes no hipMalloc, hipFree or other
 * allocating call.  At most 65536 faces per call (DSP_EINVAL beyond).  The
 * array's device address is looked up once per device on the first call
 * (hipGetSymbolAddress).  Every call on one GPU uses the same array: calls
 * that overlap on one GPU (several host threads) race and must be
 * serialised by the caller.  Synchronous (returns after the copy back).
 * Errors: DSP_EINVAL, DSP_EHIP. */
int dsp_hlld_faces_noalloc(int32_t prec, const double* wl, const double* wr, const double* bn,
                           int64_t nface, double gamma, double* flux8);

/* Free every device allocation of the set (NULL is a no-op). */
void dsp_destroy(dsp_set* set);

/* Message of the last error on the calling thread ("" if none). */
const char* dsp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
