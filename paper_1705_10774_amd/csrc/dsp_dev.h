// dsp_dev.h -- device-visible descriptions of a patch set and of the work
// buffers of one launch sequence.  Plain structs of device pointers, passed
// to kernels by value.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Makes a per-lane value opaque to the optimiser at this point (no code is
// emitted), so that what is derived from it afterwards is recomputed rather
// than hoisted and held across long stretches of the kernel.
#ifndef DSP_OPAQUE
#define DSP_OPAQUE(x) asm volatile("" : "+v"(x))
#endif

namespace dsp {

enum : int { ERR_NONFINITE = 1, ERR_NEGATIVE = 2, ERR_KMAX = 4, ERR_STATE = 8, ERR_TIMEOUT = 16 };

// A box of guard elements of one patch that take their values from one
// source patch.  Indices are the patch's own padded indices (inclusive);
// same = 1: equal resolution, source index = own index + shift; same = 0:
// resampled across resolutions, wrap = lattice shift of the periodic image.
// direct = 1 (resampled boxes only): the box exceeds the per-axis tables or
// the LDS staging of the guard-resampling kernel and is resampled straight
// from the source slices by a kernel of its own.
struct GBox {
  int lo[3], hi[3];
  int q;
  int same;
  int shift[3];
  int direct;
  int64_t wrap[3];
};

// limits of the staged guard resampling (see k_gfill): target indices per
// axis of a box, source indices a target index overlaps per axis, LDS bytes
// of staged source values
constexpr int GMAXT = 72;
constexpr int GMAXC = 4;
constexpr int GSTAGE_BYTES = 16384;

// Per-axis overlap table entry of one target index of a resampled box: the
// first overlapped source index, the number of overlapped indices, their
// normalised weights and the offsets of the overlap centres from the source
// cell centres in source cells (along a face field's own axis: the two
// bracketing source faces and their linear weights, offsets 0).
template <class T> struct GTab {
  int i0, cnt;
  T w[GMAXC], off[GMAXC];
};

// One work item of the guard resampling: a chunk of the target elements of
// box m whose source block (slope neighbours included) fits the LDS stage,
// or (tab[0] < 0) a whole same-resolution box of a padded region, copied.
// The chunk spans target indices [ta, tb] along axis ca and the whole box
// along the other two, variables [v0, v0 + nv); its staged source indices
// are r0 .. r1 per axis.  tab[d]: pool entry of target index 0 of the box's
// axis-d table.  Planned on the host at create (the geometry is static).
// The first word is m (read first when the item is prefetched).
struct GItem {
  int m, comp;
  int ca, ta, tb, v0, nv;
  int r0[3], r1[3];
  int tab[3];
  int nq;  // cells per edge of the source patch
};

// Largest tile edge of the step kernels (output cells): a patch of n cells
// per edge is cut into ceil(n / MT)^2 column tiles.
constexpr int MT = 16;

struct Bracket;

struct DevSet {
  int npatch, nslots, kmax, dt_mode, exact_time, klog_cap;
  double gamma, courant, dt_base, dt_fixed, p_floor;
  double grace;  // g of Eq. (1) (LOCAL mode)
  // non-ideal MHD (Sec. 4.3): Ohmic resistivity, ambipolar drift coefficient,
  // ion density; nonideal = eta > 0 or gamma_ad > 0
  double eta, gamma_ad, rho_i;
  int nonideal;
  int torder;  // guard time interpolation: 1 linear, 2 quadratic (three slices)
  // geometry
  const int* n;           // interior cells per edge
  const double* dx;       // cell size
  const int64_t* lo;      // lattice origin [3 * npatch]
  const int64_t* len;     // lattice edge length
  const int64_t* dxl;     // lattice cell size
  const int64_t* slot_off;   // element offset of slot 0 of each patch
  const int64_t* slice_len;  // values per slice
  const int8_t* frozen;      // boundary patch: never updated, its slice holds at every time
  // time bookkeeping (FP64 + integer ticks)
  int* cur;
  int64_t* ticks;
  double* tcur;
  int64_t* sticks;  // [npatch * nslots]
  double* stime;
  int8_t* svalid;
  // schedule record
  int64_t* steps;
  uint64_t* khash;
  int8_t* klog;  // [npatch * klog_cap]
  // readiness scan order: patch ids by decreasing n (ties by id)
  const int* scan_order;
  // neighbours (Eq. (1)) and guard boxes
  const int* nb_off;
  const int* nb_idx;
  const int* rbox_off;  // [npatch * 108 + 1]: boxes of (patch, component + 1, region)
  const GBox* boxes;
  // guard resampling plan: per patch its work items (gitem_off [npatch + 1]),
  // and the pool of per-axis tables (GTab<T> of the set's precision)
  const int* gitem_off;
  const GItem* gitems;
  const void* gtab;
  // reverse of the same-resolution boxes: per (source patch, component + 1)
  // the boxes that copy from it, as (box index, owning patch)
  const int* rev_off;  // [npatch * 4 + 1]
  const int2* rev;
  Bracket* brk;  // per box: its time bracket for the staged guard fill (k_brackets)
  int brk_ready;  // brk holds this round's brackets of the listed patches' boxes
  int maxbox;    // most boxes of one patch
  int any_direct;  // some resampled box is flagged direct (k_gfill_direct runs)
  // counters and error bits
  int* err;
  unsigned long long* floor_hits;
  unsigned long long* fallback;
  unsigned long long* updates;
  unsigned long long* algo_bytes;  // algorithmic HBM bytes of the step launches
  // device-counted rounds: when set, the ready list's length (written by the
  // readiness scan) bounds every round kernel, and rounds counts the
  // non-empty rounds
  const int* live;
  int* rounds;
  // largest ready list of a round (0: no limit); the round kernels are then
  // launched for at most scan_cap entries
  int scan_cap;
  // output cadence (Sec. 3E): a patch whose new time is a multiple of
  // out_ticks copies its new slice into frame (ticks / out_ticks - 1) mod
  // out_nframes of out_frames (host layout, host_off[p] values into the
  // frame, out_words 32-bit words per value); out_frames null: off
  void* out_frames;
  int64_t out_ticks;
  int out_nframes;
  int out_words;
  int64_t out_frame_values;
  const int64_t* host_off;
};

// Frame of patch p's output at its new time ticks, or -1: no output then.
__device__ __forceinline__ int output_frame(const DevSet& S, int64_t ticks) {
  if (!S.out_frames || ticks <= 0 || ticks % S.out_ticks != 0) return -1;
  return (int)((ticks / S.out_ticks - 1) % S.out_nframes);
}

// Copy of the current slice of patch p into output frame f by the threads
// [tid, nthr) of a group.
__device__ inline void output_copy(const DevSet& S, int p, int f, const void* slots, int tid, int nthr) {
  const int64_t w = S.out_words;
  const int64_t nw = S.slice_len[p] * w;
  const uint32_t* src = (const uint32_t*)slots + (S.slot_off[p] + (int64_t)S.cur[p] * S.slice_len[p]) * w;
  uint32_t* dst = (uint32_t*)S.out_frames + ((int64_t)f * S.out_frame_values + S.host_off[p]) * w;
  for (int64_t e = tid; e < nw; e += nthr) dst[e] = src[e];
}

// entries of a round launch: the host's count, or the device-counted length
// of the ready list when the rounds run without host round trips
__device__ __forceinline__ int live_count(const DevSet& S, int count) {
  if (!S.live) return count;
  const int m = *S.live;
  return m < count ? m : count;
}

// Courant-like factor of the Ohmic and ambipolar step limits, C_Ohm = C_AD
// (Eqs. dtOhm and dtAD).
constexpr double kCourantNonideal = 0.1;

// Work buffers of a batch of patch slots (stride = values per slot).
template <class T> struct WorkPtr {
  T* pad;   // guard-filled padded patch: 5 N^3 + 3 N^2 (N + 1)
  int64_t pad_stride;
  T* w;     // primitives, 8 N^3
  T* h;     // half-step primitives, 8 N^3
  int64_t w_stride;
  T* s;     // slopes, 3 x 8 N^3
  int64_t s_stride;
  T* f;     // fluxes, 3 x 8 (N+1)^3
  int64_t f_stride;
  int64_t fm3;  // (N+1)^3
  T* e;     // edge EMFs, 3 (N+1)^3
  int64_t e_stride;
  double* smax;  // Courant rate per slot
};

// Step of each list entry.
struct StepPtr {
  int* k;
  int64_t* dtk;
  double* dt;
};

// Device ready queue of the persistent dispatcher (k_persist): a ring of
// patch ids (id + 1; 0 = empty slot) filled by tickets, and per-patch
// ownership (0: idle, 1: queued or being updated).  Every field is written
// by the seed kernels before the persistent launch and then only through
// agent-scope atomics.
struct QueueState {
  int* buf;               // ring of cap entries
  int cap;
  unsigned* head;         // tickets taken by workers
  unsigned* tail;         // tickets given to pushed patches
  int* state;             // [npatch] ownership
  int* done;              // patches that reached the end time
  int* remaining;         // patches the advance has to bring to the end time
  int* finished;          // 1 once done == remaining
  const int64_t* tend;    // end time (ticks), written before each launch
  uint64_t timeout;       // limit of every wait, in s_memrealtime ticks (100 MHz)
};

// Level k of a local step (dt = dt_base 2^-k) from the patch Courant rate.
__device__ inline int level_for(const DevSet& S, double smax, int64_t ticks) {
  // k_c = 0 if r <= 1 else ceil(log2 r) exactly (frexp), r = dt_base smax / C;
  // raised so that the step keeps the patch time a multiple of the step
  const double r = S.dt_base * smax / S.courant;
  int kc = 0;
  if (r > 1.0) {
    int e;
    const double m = frexp(r, &e);
    kc = (m == 0.5) ? e - 1 : e;
  }
  int k = kc;
  if (ticks != 0) {
    const int tz = __ffsll((unsigned long long)ticks) - 1;
    const int al = S.kmax - tz;
    k = k > al ? k : al;
  }
  return k;
}

template <class T>
void launch_update(const DevSet& S, const int* list, int count, int nmax, T* slots, const WorkPtr<T>& W,
                   const StepPtr& st, hipStream_t s, int dt_kind, double t_end, int clip,
                   hipEvent_t ev0, hipEvent_t ev1);
// returns 1 when the Courant rate and level were computed inside the step kernel
template <class T>
int launch_fused(const DevSet& S, const int* list, int count, int nmin, int nmax, T* slots, T* pad,
                  int64_t pad_stride, bool gfill, double* smax, const StepPtr& st, hipStream_t s, int dt_kind,
                  double t_end, int clip, hipEvent_t ev0, hipEvent_t ev1);
// Persistent dispatcher (single-precision sets of one-tile patches, no
// grace): clears the queue (grid over max(cap, npatch)), then seeds it with
// the patches ready at the start; k_persist runs with `workers` workgroups
// until every patch has reached *Q.tend.  fn: 16 for sets of equal 16^3
// patches without resampled guard regions, else 0; multi: some patch has
// more than one tile (a worker then runs its tiles in turn).
void launch_queue_seed(const DevSet& S, const QueueState& Q, hipStream_t s);
void launch_persist(const DevSet& S, const QueueState& Q, float* slots, float* pad, int64_t pad_stride,
                    const StepPtr& st, int workers, int fn, bool multi, bool gfill, hipStream_t s);
template <class T>
void launch_adjoint_step(const DevSet& S, const int* list, int count, int nmax, const WorkPtr<T>& W,
                         const WorkPtr<T>& L, const StepPtr& st, const T* lam_next, T* lam_prev,
                         const int64_t* host_off, hipStream_t s);
void launch_brackets(const DevSet& S, const int* list, int count, hipStream_t s);
void launch_dt(const DevSet& S, const int* list, int count, const StepPtr& st, const double* smax, hipStream_t s,
               int dt_kind, double t_end, int clip);
void launch_publish(const DevSet& S, const int* list, int count, const StepPtr& st, hipStream_t s,
                    const void* slots = nullptr);
void launch_reset_times(const DevSet& S, unsigned long long* cnt, hipStream_t s);
void launch_scan(const DevSet& S, int64_t T_end, int* list, int* counters, hipStream_t s, int* clear = nullptr);
template <class T> void launch_stats(const DevSet& S, const T* slots, double* out, hipStream_t s);
template <class T>
void launch_gather(const DevSet& S, const T* slots, double* dst, const int64_t* host_off, hipStream_t s);
template <class T>
void launch_scatter(const DevSet& S, T* slots, const double* src, const int64_t* host_off, hipStream_t s);
template <class T>
void launch_pack(const DevSet& S, const T* slots, T* dst, const int64_t* host_off, hipStream_t s);
template <class T> void launch_poison(const DevSet& S, T* slots, hipStream_t s);
template <class T>
void launch_hlld_faces(const double* wl, const double* wr, const double* bn, int64_t nface, double gamma, double* out,
                       hipStream_t s);
template <class T>
void launch_unpack(const DevSet& S, T* slots, const T* src, const int64_t* host_off, hipStream_t s);

}  // namespace dsp
