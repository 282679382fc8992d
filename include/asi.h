/*
 * asi.h -- C ABI of the MI355X (gfx950) artificial-spin-ice relaxation library.
 *
 * The library runs the flatspin dipole model (Jensen et al., "flatspin: A
 * Large-Scale Artificial Spin Ice Simulator") on the GPU:
 *   - dipole-dipole field on every magnet from its neighbours within the
 *     neighbour distance (Sec. II.C, Eq. 3), projected on each magnet's easy
 *     (parallel) and hard (perpendicular) axis, plus the global applied field
 *     (Sec. II.D) and a per-step thermal field (Sec. II.E) -- Eq. 2;
 *   - the generalized Stoner-Wohlfarth switching test (Sec. II.F, Eq. 5 and
 *     Eq. 6) with per-magnet coercive fields h_k (Sec. II.G);
 *   - deterministic single-spin-flip relaxation (Sec. II.H): flip the
 *     flippable magnet with the greatest Eq. 5 left-hand side (ties: lowest
 *     index), update its neighbours, repeat until none can flip, then take
 *     the next field step.
 * All model arithmetic is FP64.  Spins are int8 (+1 / -1).
 *
 * Conventions for every entry point:
 *   - Every call returns an asi_status; nothing throws across the ABI.
 *     asi_last_error() describes the last failure on the calling thread.
 *   - Input arrays are copied before the call returns; the caller keeps
 *     ownership and may free them at once.  Output arrays are allocated by
 *     the caller, host memory, with the element counts stated below.
 *   - A handle owns all of its device memory and uses one HIP stream.  Calls
 *     that return results synchronise that stream first.  A handle is not
 *     thread-safe; distinct handles may be driven from distinct threads.
 *   - After a HIP error (ASI_EDEVICE) the handle is poisoned: later calls on
 *     it return ASI_ESTATE; only asi_destroy remains valid.
 *   - Positions are in units of the lattice spacing, angles in radians.
 */
#ifndef ASI_H
#define ASI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct asi_sim* asi_handle;

typedef enum {
  ASI_OK = 0,
  ASI_EINVAL = -1,   /* bad argument, coincident magnets, step out of range */
  ASI_ENOMEM = -2,   /* allocation failed or HBM budget exceeded            */
  ASI_EDEVICE = -3,  /* HIP runtime error; the handle is poisoned            */
  ASI_ESTATE = -4,   /* handle poisoned, or call invalid in this state       */
  ASI_ELOOP = -5,    /* a relax exceeded max_flips_per_step                  */
  ASI_EBUSY = -6     /* server: job not finished yet                         */
} asi_status;

/* Device memory and stream plumbing.  With alloc == NULL the library uses
 * hipMalloc / hipFree itself.  With callbacks, every device allocation of
 * the handle goes through them (for example PyTorch's caching allocator),
 * stream-ordered on `stream`.  stream == NULL: the library creates its own
 * (default priority) stream. */
typedef struct {
  void* stream;                                            /* hipStream_t */
  void* (*alloc)(size_t bytes, void* stream, void* ctx);   /* NULL on failure */
  void (*free)(void* ptr, void* stream, void* ctx);
  void* ctx;
} asi_device;

/* One simulation instance (Sec. II).  struct_size = sizeof(asi_params). */
typedef struct {
  uint32_t struct_size;
  int64_t n;                 /* magnets, 1 <= n < 2^31                          */
  const double* xy;          /* [2n] positions (x0, y0, x1, y1, ...), distinct  */
  const double* theta;       /* [n] island rotation: mhat = (cos, sin)(theta)   */
  const int8_t* spin0;       /* [n] start spins +-1, or NULL => all +1          */
  const double* hk;          /* [n] coercive field h_k^(i) > 0 (Sec. II.G), or
                                NULL => drawn from hk_mean, k_disorder below  */
  double alpha;              /* dipolar coupling strength of Eq. 3, finite      */
  double neighbor_distance;  /* d >= 0: j is a neighbour of i iff
                                (x_i-x_j)^2 + (y_i-y_j)^2 <= (d + 1e-9)^2      */
  double b, c, beta, gamma;  /* generalized astroid of Eq. 5, all > 0; b, beta,
                                gamma finite.  c may be +INFINITY: the hard-axis
                                term of Eq. 5 vanishes, and with b = 1, gamma
                                = 2 the test becomes the parallel-only
                                criterion -s_i h_par > h_k^(i) (Sec. IV.C)    */
  double thermal_std;        /* sigma_th >= 0 of Sec. II.E; 0 => no thermal     */
  uint64_t thermal_seed;     /* Philox4x32-10 key (lo, hi 32 bits)              */
  int64_t max_flips_per_step;/* 0 => 64 * n; a relax exceeding it => ASI_ELOOP  */
  int64_t flip_log_capacity; /* entries kept in the flip log; 0 => 4n + 65536.
                                Flips beyond it are counted and hashed only.    */
  int32_t field_mode;        /* how a magnet's dipolar sum (Eq. 3) is obtained at
                                each field step:
                                0 (default) carry: gathered once, then updated
                                  by every neighbour flip across steps;
                                1 dirty: re-gathered in ascending neighbour
                                  order when a neighbour flipped since;
                                2 full: re-gathered for every magnet every step.
                                1 and 2 give bitwise identical results and
                                fields that are a function of the spins only;
                                0 differs from them by rounding.               */
  /* Disorder of Sec. II.G, used when hk == NULL: h_k^(i) = hk_mean +
     (k_disorder * hk_mean) * z_i, z_i the first Box-Muller normal of
     Philox4x32-10 keyed (disorder_seed lo, hi) at counter (i, 0, 1, 0)
     (u1, u2 formed as for the thermal field); draws below 1e-12 * hk_mean
     are raised to it.  hk_mean > 0, k_disorder >= 0, both finite. */
  double hk_mean;
  double k_disorder;
  uint64_t disorder_seed;
} asi_params;

/* Build an instance: copies the inputs, builds the neighbour lists and the
 * projected coupling tensors on the device (Sec. II.C).  The current step is
 * -1 (no applied and no thermal field) until the first asi_run. */
asi_status asi_create(const asi_params* params, const asi_device* dev, asi_handle* out);

/* Set the external-field time series (Sec. II.D): h_xy[2*k], [2*k+1] is the
 * global field (x, y) of step k, 0 <= k < n_steps.  Copied. */
asi_status asi_set_field_protocol(asi_handle h, int64_t n_steps, const double* h_xy);

/* Per-magnet external field (Sec. II.D), added to the global H[t] of every
 * step: the external field of magnet i at step t is H[t] + h_loc(i, t), with
 * h_loc(i, t) = (h_loc[2*(k*n + i)], h_loc[2*(k*n + i) + 1]) and k = 0 when
 * n_slabs == 1 (a static local or spatial field, e.g. a gradient sampled at
 * the positions), k = t when n_slabs equals the protocol length (a local
 * time series).  n_slabs == 0 removes it.  Copied to the device (16 * n *
 * n_slabs bytes), host memory; ASI_EINVAL for any other n_slabs, a NULL
 * h_loc with n_slabs > 0 or a non-finite value.  While a series (n_slabs >
 * 1) is set, asi_set_field_protocol accepts only the same length. */
asi_status asi_set_local_field(asi_handle h, int64_t n_slabs, const double* h_loc);

/* Travelling-wave local field evaluated in the field pass (Sec. II.D), no
 * per-step storage: magnet i at step t gets
 *   amp * sin(2 pi (kx x_i + ky y_i) + phase0 - 2 pi t / period_steps) * (cos angle, sin angle)
 * added to H[t] and to any asi_set_local_field field.  xy: host [2n], the
 * instance's positions (8 bytes per magnet are kept on the device).  All
 * values finite, period_steps != 0; amp == 0 removes the wave. */
asi_status asi_set_local_wave(asi_handle h, const double* xy, double amp, double kx, double ky,
                              double period_steps, double phase0, double angle);

/* Thermal schedule (Sec. II.E; the annealing protocols of Sec. IV.B): step t
 * draws its thermal field with standard deviation sigma[t] instead of
 * thermal_std (same normals: Philox counter (i, t, 0, 0)), so a constant
 * schedule equals that constant thermal_std bit for bit.  n_steps must equal
 * the protocol length; 0 returns to thermal_std.  Copied; host memory;
 * ASI_EINVAL for another length, a NULL sigma or a negative or non-finite
 * value.  While set, asi_set_field_protocol accepts only the same length. */
asi_status asi_set_thermal_schedule(asi_handle h, int64_t n_steps, const double* sigma);

/* Net magnetisation of the current spins, M = sum_i s_i mhat_i (Eq. 1
 * summed; a hysteresis loop plots M . Hhat / M_S with M_S = n, Sec. IV),
 * reduced on the device in a fixed order: the same spins give the same bits.
 * m_out: host double[2] (x, y). */
asi_status asi_magnetization(asi_handle h, double* m_out);

/* Net magnetisation of groups of magnets, e.g. the islands that meet at each
 * vertex (the vertex maps of Sec. IV.B): group g is idx[ptr[g] .. ptr[g+1])
 * (CSR, host arrays, ptr[0] = 0, non-decreasing, 0 <= idx < n), and out[2g],
 * out[2g+1] (host) receive sum s_i mhat_i over it, added in that order.
 * ASI_EINVAL for malformed groups (checked before any device work). */
asi_status asi_group_magnetization(asi_handle h, int64_t n_groups, const int64_t* ptr,
                                   const int32_t* idx, double* out);

/* Spin-spin correlation by separation (Sec. IV.B), over the neighbour pairs
 * of the instance (Sec. II.C), each pair once.  A pair correlates +1 when its
 * dipolar energy -s_i s_j A_ij is minimal (s_i s_j A_ij > 0, A_ij the
 * coupling along the easy axes), -1 when maximal, 0 when the coupling is
 * zero up to rounding (|A_ij| <= 1e-9 |alpha| / r^3).  Pair (i, j) at
 * distance r = sqrt(dx^2 + dy^2) (each operation correctly rounded, dx =
 * x_i - x_j) goes to bin floor(r / bin_width) when that is < n_bins.
 * xy: host [2n], the positions the instance was created with.  Outputs (host
 * int64[n_bins]): sum_out the summed correlations, count_out the pairs; the
 * mean correlation of bin b is sum_out[b] / count_out[b].  1 <= n_bins <=
 * 4096; bin_width finite > 0. */
asi_status asi_spin_correlation(asi_handle h, const double* xy, double bin_width,
                                int32_t n_bins, int64_t* sum_out, int64_t* count_out);

/* Switching order (Sec. IV.D): pos_out[j] (host int64[n]) receives the
 * position in the flip log (0-based, counting from create / set_state) of
 * magnet j's first switch, or the log's length for a magnet that never
 * switched.  Computed on the device from the flip log.  ASI_ESTATE when
 * more flips happened than flip_log_capacity keeps. */
asi_status asi_switching_order(asi_handle h, int64_t* pos_out);

/* Spearman's rank correlation coefficient rho of the switching orders of
 * two instances of the same n magnets (Sec. IV.D; e.g. the same array at two
 * lattice spacings, or with and without coupling): the Pearson correlation
 * of the two vectors of ranks of the asi_switching_order positions, tied
 * positions (magnets that never switched) sharing their mean rank.  On the
 * device, exactly: with u_i = 2 rank_i - (n + 1) (an integer), the sums
 * Sab = sum u_a u_b, Saa = sum u_a^2, Sbb = sum u_b^2 are formed in integer
 * arithmetic, then rho = Sab / sqrt(Saa * Sbb) in FP64 from the totals
 * rounded to double (NaN when Saa or Sbb is 0).  sums_out (may be NULL):
 * int64[6], the three totals as 128-bit two's complement (low, high) pairs.
 * a == b is allowed (rho = 1 unless every magnet ties).  ASI_EINVAL for
 * different n or n outside 2 .. 2^27; ASI_ESTATE as asi_switching_order. */
asi_status asi_switching_rho(asi_handle a, asi_handle b, double* rho_out, int64_t* sums_out);

/* asi_switching_rho for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same rho and sums, bit for bit, with no hipMalloc, hipFree
 * or allocator callback.  Its working memory is one static device array per
 * GPU (about 33 MB, held until the process ends), found with
 * hipGetSymbolAddress on the first call on each GPU.  Limits: n in 2 .. 2^20
 * and at most 2^24 flips in each instance's log, else ASI_EINVAL; both
 * handles on the same GPU.  Every call on a GPU shares that GPU's array:
 * calls are serialised within the process by a lock and each synchronises
 * before returning, and no call depends on what an earlier one left there;
 * a call that overlapped another on the same array (another copy of the
 * library in the same process) would race.  Errors as asi_switching_rho. */
asi_status asi_switching_rho_noalloc(asi_handle a, asi_handle b, double* rho_out,
                                     int64_t* sums_out);

/* Per-step magnetisation log: while enabled, asi_run and asi_relax record M
 * after the relax of every step t they run into row t of a device array of
 * the protocol's length (rows of steps not run hold NaN; a new protocol
 * clears it).  Batched and served runs do not record.  enable = 0 frees it. */
asi_status asi_set_magnetization_log(asi_handle h, int32_t enable);

/* Copy the log: out = host double[n_steps][2].  ASI_ESTATE when it is off. */
asi_status asi_get_magnetization_log(asi_handle h, double* out);

/* Relax under the current step's fields (Sec. II.H) without advancing t.
 * flips_out (may be NULL) receives the number of flips of this call. */
asi_status asi_relax(asi_handle h, int64_t* flips_out);

/* The time loop of Sec. II.H: for t = t_begin .. t_end-1, set the fields of
 * step t (applied H[t] of Sec. II.D and the thermal draw of Sec. II.E, both
 * held fixed while the step relaxes) and relax to stability.  Requires 0 <= t_begin <= t_end <=
 * n_steps.  flips_out (may be NULL): flips of this call.  Stops early with
 * ASI_ELOOP when one step exceeds max_flips_per_step. */
asi_status asi_run(asi_handle h, int64_t t_begin, int64_t t_end, int64_t* flips_out);

/* Current state: spins s_i of Eq. 1 [n], the total field of Eq. 2
 * projected on the easy axis h_par [n] and hard axis h_perp [n] (the two
 * components the astroid of Eq. 5 reads, Sec. II.F) as of the end of the
 * last relax, and the last completed step (-1 if none).  Any pointer may be
 * NULL. */
asi_status asi_get_state(asi_handle h, int8_t* spins, double* h_par, double* h_perp,
                         int64_t* step_out);

/* Overwrite the spins [n] (+-1) and the current step (-1 .. n_steps-1),
 * e.g. to resume from a checkpoint taken at a step boundary.  Every dipolar
 * sum is re-gathered from the spins at the next field step, so with
 * field_mode 1 or 2 a resumed run is bitwise identical to an uninterrupted
 * one; with field_mode 0 the carried sums it replaces differ from the
 * re-gathered ones by rounding only.  Resets the flip log and its hash. */
asi_status asi_set_state(asi_handle h, const int8_t* spins, int64_t step);

/* Flip log of the relax of Sec. II.H, one entry per switching event of
 * Sec. II.F in the order the relax performed them: the first
 * min(count, cap, flip_log_capacity) flips as (step, magnet index), the
 * total number of flips logged since create / set_state, and a running hash
 * over all of them: hash = 0xcbf29ce484222325, then for each flip
 * hash = (hash ^ ((uint64)(uint32)step << 32 | (uint32)index)) * 0x100000001b3
 * modulo 2^64.  step and idx may be NULL when cap == 0. */
asi_status asi_get_flip_log(asi_handle h, int64_t cap, int32_t* step, int32_t* idx,
                            int64_t* count_out, uint64_t* hash_out);

/* Per-step flip counts of the protocol's steps [0, n_steps) (counts of the
 * most recent run of each step).  out: [n_steps] int32. */
asi_status asi_get_step_flips(asi_handle h, int32_t* out);

/* Evaluate the fields of step t (-1 .. n_steps-1) for the current spins --
 * one full-field pass over every magnet (Eq. 2, Eq. 3 projected) -- without
 * relaxing.  Results are read back with asi_get_state. */
asi_status asi_compute_fields(asi_handle h, int64_t t);

typedef struct {
  int64_t n;                /* magnets                                          */
  int64_t n_edges;          /* directed neighbour pairs E                        */
  int32_t max_degree;       /* padded row length of the neighbour tables         */
  int32_t relax_waves;      /* wavefronts of the relax workgroup                 */
  int64_t device_bytes;     /* device memory held by the handle                  */
  double field_pass_bytes;  /* algorithmic bytes of one full-field pass:
                               20 per neighbour pair + 53 per magnet, + 16
                               per magnet with a local field set, + 8 with a
                               local wave                                     */
  int64_t flip_log_capacity;/* flip-log entries kept (asi_params)               */
} asi_info;
asi_status asi_get_info(asi_handle h, asi_info* out);

/* Kernel timing with HIP events on the handle's stream (off by default).
 * Totals accumulate from the call that enables timing. */
typedef struct {
  int64_t field_launches;   double field_ms;   /* full-field pass kernel */
  int64_t relax_launches;   double relax_ms;   /* relax kernel           */
} asi_timing;
asi_status asi_set_timing(asi_handle h, int32_t enable);
asi_status asi_get_timing(asi_handle h, asi_timing* out);

/* Launch shapes of the relax (Sec. II.H); any valid choice gives the same
 * flips, log and fields, bit for bit -- only the speed differs. */
typedef struct {
  int32_t relax_waves;  /* wavefronts per relax workgroup, 1..16 (the
                           speculative path needs 16)                       */
  int32_t l1_shift;     /* log2 of the relax tree's first-level tile, from
                           the handle's minimum (tiles <= 2048) up to 20     */
  int64_t spec_min;     /* flippable magnets at a step's start for the
                           speculative path, >= 1 (it also needs a degree
                           <= 128)                                           */
  double default_ms;    /* asi_tune: sample time with the shapes it found    */
  double tuned_ms;      /* asi_tune: sample time with the shapes it chose    */
  int32_t trials;       /* asi_tune: shapes timed (0: taken from the cache)  */
  int32_t field_rows;   /* rows per workgroup of the full-field pass at >= 128
                           neighbours (field_mode 2): 8, 16, 32 or 64; 0 =
                           chosen by the instance size (below 256 slices of
                           64 rows: split over the 64-slot chunks)          */
} asi_tuning;
/* Autotuner: times the next sample_steps (>= 1, clipped to the protocol)
 * field steps under candidate shapes (rows per workgroup of the
 * high-degree full-field pass, speculation threshold, then tile size, then
 * workgroup size), each run from a device snapshot of the handle's state,
 * and keeps the fastest.  The result is cached per (GPU architecture,
 * floor(log2 n), floor(log2 max_degree), field_mode): a later call on a
 * handle of the same class applies the cached shapes without timing
 * (trials = 0).  ASI_TUNE_CACHE=<file> keeps the cache in a text file
 * across processes; ASI_TUNE_NOCACHE=1 always times.  Every trial must reproduce the
 * first trial's flip count and hash, else ASI_ESTATE.  The state, cursor
 * and flip log are restored exactly; out (may be NULL) receives the choice.
 * The snapshot is allocated through the handle's device allocator.
 * ASI_ESTATE without a protocol, ASI_EINVAL if no step is left to sample. */
asi_status asi_tune(asi_handle h, int64_t sample_steps, asi_tuning* out);
/* Current shapes (the *_ms and trials fields are 0). */
asi_status asi_get_tuning(asi_handle h, asi_tuning* out);
/* Set shapes, e.g. from an earlier asi_tune; ASI_EINVAL if out of range. */
asi_status asi_set_tuning(asi_handle h, const asi_tuning* t);

asi_status asi_destroy(asi_handle h);

/* Thread-local description of the last failure; valid until the next call
 * on this thread. */
const char* asi_last_error(void);

/* ---- batching: many independent instances in few launches -------------
 * Runs every handle from its current step to the end of its own protocol.
 * All handles must live on the same device; the work runs on a stream of
 * its own.  Each instance's flips, spins and fields are bitwise identical to
 * running it alone with asi_run.  flips_out: [count] or NULL.
 *   mode 0: per field step, one field launch over all instances and one
 *           relax launch (a workgroup per instance);
 *   mode 1: the same pair captured once in a HIP graph, replayed per step;
 *   mode 2: one field launch, then one persistent launch in which each
 *           instance's workgroup runs all of its remaining steps (field phase
 *           and relax) without waiting for the other instances. */
asi_status asi_batch_run(asi_handle* hs, int32_t count, int32_t mode, int64_t* flips_out);

/* ---- serving: continuous batching of arriving simulation jobs -----------
 * A server keeps up to max_slots jobs resident on the device within
 * hbm_budget_bytes, admitting queued jobs as slots and memory free up.
 * Each finished job's result is bitwise identical to a plain asi_run of the
 * same inputs. */
typedef struct asi_server* asi_server_t;
asi_status asi_server_create(const asi_device* dev, size_t hbm_budget_bytes,
                             int32_t max_slots, asi_server_t* out);
/* Queue a job: instance parameters plus its protocol (copied).  job_id_out
 * receives a non-negative id.  ASI_ENOMEM if the job alone exceeds the
 * budget. */
asi_status asi_server_submit(asi_server_t s, const asi_params* p, int64_t n_steps,
                             const double* h_xy, int64_t* job_id_out);
/* The same with the per-magnet external field of asi_set_local_field
 * (loc_slabs 0, 1 or n_steps; h_loc host [loc_slabs][n][2]) and the thermal
 * schedule of asi_set_thermal_schedule (sigma host [n_steps], or NULL for
 * thermal_std), copied and applied at admission; the footprint counts them. */
asi_status asi_server_submit_fields(asi_server_t s, const asi_params* p, int64_t n_steps,
                                    const double* h_xy, int64_t loc_slabs, const double* h_loc,
                                    const double* sigma, int64_t* job_id_out);
/* Advance the server by one burst: run every resident job for about
 * budget_ms of device time (each job's workgroup advancing through its own
 * protocol; a relax still running at the deadline pauses mid-step and
 * resumes where it stopped), admit queued jobs that fit while the burst runs
 * (neighbour tables built at admission; they join the next burst), then
 * retire finished ones.  With at most 8 jobs resident, one of them large
 * (>= 2^17 magnets), the burst is a sequence of rounds instead, each a field
 * pass spread over the whole device and one relax step of every job.
 * active_out (may be NULL): jobs still queued or resident. */
asi_status asi_server_step(asi_server_t s, double budget_ms, int32_t* active_out);
/* done_out = 1 when the job has finished (non-blocking). */
asi_status asi_server_poll(asi_server_t s, int64_t job_id, int32_t* done_out);
/* Result of a finished job: spins [n] (may be NULL), flip count and hash,
 * and host clock seconds at admission and completion.  ASI_EBUSY if not
 * finished.  The job's memory is released on take. */
asi_status asi_server_take(asi_server_t s, int64_t job_id, int8_t* spins, int64_t* flips,
                           uint64_t* flip_hash, double* t_admit, double* t_done);
/* Counters since the server was created.  Host seconds are wall time of
 * the calling thread; admit_s overlaps device bursts. */
typedef struct {
  int64_t bursts;    /* device bursts launched                                 */
  int64_t admitted;  /* jobs created on the device                             */
  int64_t retired;   /* jobs that finished on the device (done or ELOOP)       */
  int64_t pauses;    /* relaxes stopped at a burst deadline, resumed later      */
  double admit_s;    /* creating admitted jobs                                 */
  double wait_s;     /* waiting for bursts after admission                     */
  double retire_s;   /* reading results back and releasing jobs                */
  double rebuild_s;  /* rebuilding the launch tables after admissions/retires  */
} asi_server_stats;
asi_status asi_server_get_stats(asi_server_t s, asi_server_stats* out);
asi_status asi_server_destroy(asi_server_t s);

/* ---- measurement aid (not part of the model) ---------------------------
 * Latency of dependent global-memory loads, the floor of the relax of Sec.
 * II.H, whose flips are chains of such loads: lanes 1 .. 64 of one
 * wavefront each follow a pointer chain through a buffer of `bytes` bytes
 * (one 4-byte element per 128-byte line, the lines in one random cycle drawn
 * from `seed`, built and checked on the host; lane l starts l/64 of the way
 * round), `hops` loads each, timed with the device's constant-rate clock,
 * after a first untimed pass (the whole cycle for buffers of at most 64 MiB,
 * else `hops` loads per lane) that the timed pass continues.
 * With lanes = 1 a hop is one load; with 64 it is one scattered 64-address
 * gather.  A buffer that fits the L2 (a few MB) gives the L2 latency; in one
 * far beyond the 256 MB last-level cache every timed load is to a line not
 * touched before, which gives the HBM latency (address translations warm).  ns_out receives
 * nanoseconds per hop.  Allocates bytes / 32 bytes through dev (NULL:
 * hipMalloc on the current device, own stream).  ASI_EINVAL unless hops >=
 * 1, 1 <= lanes <= 64 and 8 KiB <= bytes <= 2^36. */
asi_status asi_measure_load_latency(const asi_device* dev, int64_t bytes, int64_t hops,
                                    int32_t lanes, uint64_t seed, double* ns_out);

#ifdef __cplusplus
}
#endif
#endif /* ASI_H */
