/*
 * pmf.h -- C ABI of the MI355X spectral point-mass filter library (libpmf.so).
 *
 * The library carries grid-based probability densities of the state of a linear
 * SDE  dx = A x dt + Q dw  (E[dw dw^T] = I dt; Sec. I, eq. dynam) through
 *   - the time update: the Fokker-Planck equation of Sec. I.B (eq. fokker) on a
 *     grid that moves with x' = A x (Sec. II.B, eqs. movFPEadv / easyFPE), solved
 *     with spectral derivatives (Sec. IV, eqs. fourtrsf / interFreq / secDer;
 *     Sec. V Algorithm) on a Fourier grid, or with Chebyshev differentiation
 *     matrices (Sec. IV.B) on a Chebyshev grid;
 *   - the measurement update: Bayes' rule of Sec. I.A (eq. filt) with the
 *     measurement z = h(x) + v of eq. meas, the normalisation of Sec. III.A
 *     (eq. PDF_pm), then a new grid and re-interpolation onto it.
 * The diffusion matrix of the Fokker-Planck equation is D = Q Q^T.
 *
 * Conventions for every entry point:
 *   - Plain pointers and sizes only.  Host pointers are owned by the caller and
 *     are only read or written during the call (or, for `loglik`, by the
 *     asynchronous copy that the call enqueues -- see pmf_update).
 *   - Device memory is owned by the library; it is obtained through the
 *     allocator given to pmf_ctx_create (NULL = hipMalloc/hipFree).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *     marked "async" only enqueue work on it.
 *   - Errors found on the host are returned at once and leave all state as it
 *     was.  Errors found on the device (a zero or non-finite normaliser) leave
 *     the density and grid as they were and are reported by the next call that
 *     synchronises (pmf_moments, pmf_get_state, pmf_sync_status).
 *   - No C++ exception crosses this boundary.  One filter must not be used by
 *     two threads at once; distinct filters and contexts are independent.
 *   - pmf_last_error() returns a thread-local message for the last failure.
 *
 * Density layout in device memory: prod(N[0..nx-1]) values of the filter's
 * precision, C order (last axis fastest).  Fourier grids: node j sits at
 * x_j = c + M (j - N/2).  Chebyshev grids: x = c + M u, u_a = -cos(j_a pi/(N_a+1)),
 * j_a = 1..N_a (the interior of a Chebyshev-Gauss-Lobatto set; the density is
 * zero at u = +-1).  M's columns are the per-index step vectors (Fourier) or the
 * half-width vectors (Chebyshev).
 */
#ifndef PMF_H
#define PMF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PMF_OK = 0,
    PMF_E_INVALID = 1,     /* bad argument; nothing was changed */
    PMF_E_NOMEM = 2,       /* device allocation failed */
    PMF_E_DEVICE = 3,      /* a HIP call failed */
    PMF_E_DEGENERATE = 4,  /* a measurement update met a zero / non-finite normaliser
                              or grid; that update left density and grid unchanged */
    PMF_E_BUSY = 5,        /* server: no slot or memory for the request now */
    PMF_W_BOUNDARY = 64    /* warning bit: a posterior had more than 1e-4 of its mass
                              on the outermost layer of grid nodes */
} pmf_status;

enum { PMF_GRID_FOURIER = 0, PMF_GRID_CHEBYSHEV = 1 };
enum { PMF_INT_EXACT = 0, PMF_INT_RK4 = 1, PMF_INT_EULER = 2, PMF_INT_FDM = 3, PMF_INT_SINE = 4 };
enum { PMF_INTERP_AUTO = 0, PMF_INTERP_LAGRANGE = 1 };
enum { PMF_H_LINEAR = 0, PMF_H_CUBIC1 = 1, PMF_H_NORM = 2, PMF_H_TERRAIN = 3 };
enum { PMF_FP64 = 0, PMF_FP32 = 1 };

#define PMF_MAX_NX 4
#define PMF_MAX_MIX 4
#define PMF_MAX_TERRAIN 8

typedef struct {
    /* alloc(bytes, user, stream) -> device pointer or NULL; free(ptr, user, stream) */
    void* (*alloc)(size_t, void* user, void* stream);
    void (*free)(void*, void* user, void* stream);
    void* user;
} pmf_allocator;

/* Model of one filter (Sec. I, eqs. dynam/meas). */
typedef struct {
    int nx;                     /* state dimension, 1..4 (Chebyshev grids: 1..3) */
    double A[16];               /* row-major nx x nx drift matrix */
    double Q[16];               /* row-major nx x nx noise gain; D = Q Q^T */
    int grid;                   /* PMF_GRID_FOURIER or PMF_GRID_CHEBYSHEV */
    int N[4];                   /* points per axis.  Fourier: even, 2^a 3^b 5^c 7^d
                                   11^e 13^f 17^g, 4..256 (the fdm and sine
                                   integrators also need 2 (N + 1) of that form).
                                   Chebyshev: 4..256 */
    double span_sigmas;         /* grid half-width in standard deviations (e.g. 8) */
    double t_nominal;           /* interval used by the grid design, > 0 */
    int integrator;             /* PMF_INT_EXACT | _RK4 | _EULER | _FDM | _SINE
                                   (Chebyshev grids: RK4 only) */
    int substeps;               /* minimum number of substeps l (>= 1) */
    int precision;              /* PMF_FP64 or PMF_FP32 density; reductions are FP64 */
    int interp;                 /* PMF_INTERP_AUTO: spectral (trigonometric or
                                   Chebyshev polynomial) per axis when the old grid is
                                   axis aligned, else cubic Lagrange; PMF_INTERP_LAGRANGE:
                                   always cubic Lagrange */
    int meas_kind;              /* PMF_H_LINEAR: h = H x;  PMF_H_CUBIC1: h = a1 x1 + a3 x1^3
                                   (hparam[0], hparam[1]);  PMF_H_NORM: h = ||x||;
                                   PMF_H_TERRAIN: a smooth synthetic terrain map,
                                   h = sum_m a_m cos(w_m . x + phi_m) (the table
                                   function of Sec. VI replaced by an analytic one) */
    int nz;                     /* measurement dimension (1 for CUBIC1, NORM, TERRAIN), 1..3 */
    double H[12];               /* row-major nz x nx (PMF_H_LINEAR) */
    double hparam[4];
    int nterrain;               /* PMF_H_TERRAIN: components, 1..PMF_MAX_TERRAIN */
    double terrain[PMF_MAX_TERRAIN * 6];   /* component m at terrain[6m]: a_m, phi_m,
                                              w_m[0..nx) */
    int noise_ncomp;            /* Gaussian-mixture components of v, 1..4 */
    double noise_w[4];          /* weights (normalised by the library) */
    double noise_mean[4 * 3];   /* component g: noise_mean[3g .. 3g+nz) */
    double noise_cov[4 * 9];    /* component g: row-major nz x nz at noise_cov[9g] */
} pmf_model;

/* Gaussian-mixture prior p(x0) (Sec. I). */
typedef struct {
    int ncomp;                  /* 1..4 */
    double w[4];
    double mean[4 * 4];         /* component g at mean[4g] */
    double cov[4 * 16];         /* component g: row-major nx x nx at cov[16g] */
} pmf_prior;

/* Header of the host image written by pmf_get_state; the density follows it
 * (prod(N) values of the filter's precision, C order). */
typedef struct {
    unsigned int magic;         /* PMF_STATE_MAGIC */
    int version;                /* 2 */
    int nx, grid, precision, status;
    int N[4];
    double c[4];
    double M[16];               /* row-major, row stride 4 */
    double t;
} pmf_state_header;
#define PMF_STATE_MAGIC 0x504d4631u

typedef struct pmf_ctx pmf_ctx;
typedef struct pmf_filter pmf_filter;

/* Checks a model as pmf_create does, on the host only (no device is touched):
 * PMF_OK, or PMF_E_INVALID with the reason in pmf_last_error().  With fusable
 * not NULL, *fusable is set to 1 if pmf_batch_step accepts filters of this model
 * and to 0 otherwise, the reason then written to why (NULL, or why_len bytes). */
pmf_status pmf_model_check(const pmf_model* model, int* fusable, char* why, size_t why_len);

/* Context bound to one HIP device.  `a` may be NULL (hipMalloc/hipFree); else
 * every device allocation of the context's filters and batches goes through
 * a->alloc / a->free (e.g. a framework's caching allocator), which may be called
 * from the calling thread or from a server's threads.  The allocator struct is
 * copied. */
pmf_status pmf_ctx_create(int device, const pmf_allocator* a, pmf_ctx** out);
void pmf_ctx_destroy(pmf_ctx* ctx);

/* New filter: validates the model, designs the first grid from the prior's
 * mean and covariance (centre = mean, half-widths span_sigmas * sqrt(diag(cov +
 * W(t_nominal))), W(T) = int_0^T e^{-As} D e^{-A^T s} ds), evaluates the prior PDF
 * at the nodes and normalises (Sec. III.A).  Synchronous; uses the null stream. */
pmf_status pmf_create(pmf_ctx* ctx, const pmf_model* model, const pmf_prior* prior,
                      pmf_filter** out);
void pmf_destroy(pmf_filter* f);

/* Time update over an interval T >= 0 (Sec. I.B; Sec. V Algorithm).  Async.
 * Fourier grids: forward FFT, per-mode gain, inverse FFT; the gain is
 *   exact:  exp(-1/2 kappa^T W_y kappa),  W_y = M^-1 W(T) M^-T;
 *   rk4:    the product over l substeps of the classic RK4 amplification of
 *           lambda(t) = -1/2 kappa^T D_y(t) kappa,  D_y(t) = M(t)^-1 D M(t)^-T;
 *   euler:  the product of 1 / (1 + h/2 kappa^T D_y(t_n) kappa), n = 0..l-1
 *           (implicit diffusion, Sec. V.A);
 * times e^{-tr(A) T} (the trace term of eq. easyFPE).
 *   fdm:    the finite-difference baseline of Sec. III.B: l explicit steps of
 *           eq. FDM (step matrices of eq. fdiff per axis, the trace term inside),
 *           the nodes taken as interior nodes with zeros beyond both ends,
 *           computed by the sine-transform route of eq. FST: a fast DST-I (an
 *           FFT of the odd extension, length 2 (N_a + 1)) along every axis, the
 *           product over n of the step eigenvalues
 *           1 - h tr(A) + h sum_a D_y,aa(t_n) (cos(j_a pi / (N_a + 1)) - 1),
 *           DST-I back.  Needs diagonal A and D (Fourier grid; the designed
 *           grids are axis-aligned, so D_y stays diagonal);
 *           l = max(substeps, ceil(T max_t sum_a D_y,aa(t))) at t = 0, T/2, T.
 *   sine:   the sine-series variant of the spectral update (the non-periodic
 *           alternative named in Sec. IV's notes): DST-I along every axis, each
 *           sine mode times exp(-1/2 sum_a W_y,aa k_a^2) e^{-tr(A) T} with
 *           k_a = j_a pi / (N_a + 1) (exact in time, zero beyond both grid ends),
 *           DST-I back.  Diagonal A and D, Fourier grid, as fdm.  Mixed derivatives use the
 * first-derivative symbol (no Nyquist term), squares keep it (eq. secDer).
 * Chebyshev grids: classic RK4 with dense differentiation matrices.
 * RK4 uses l = max(substeps, ceil(T lambda_max / 2.5)) substeps; lambda_max bounds
 * 1/2 sum_ab |D_y,ab| rho_a rho_b at t = 0, T/2, T (rho = pi for Fourier axes, the
 * square root of the spectral radius of the second-derivative matrix for
 * Chebyshev axes).  Then c <- e^{AT} c, M <- e^{AT} M, t <- t + T. */
pmf_status pmf_predict(pmf_filter* f, double T, void* stream);

/* Measurement update with z[0..nz) (Sec. I.A).  Async.  log p(z_k | z^{k-1})
 * is written to *loglik by an asynchronous copy enqueued on `stream` when loglik
 * is not NULL: the caller must synchronise the stream before reading it (pinned
 * host memory keeps the copy asynchronous).  Non-finite z -> PMF_E_INVALID.
 * Steps: log-likelihood at the nodes, shift by its maximum, multiply, FP64
 * normaliser and moments, new grid (centre = posterior mean, half-widths from the
 * posterior covariance + W(t_nominal)), interpolation onto it (zero outside the
 * old grid), renormalisation.  A zero or non-finite normaliser leaves the filter
 * unchanged and sets PMF_E_DEGENERATE in its status word. */
pmf_status pmf_update(pmf_filter* f, const double* z, double* loglik, void* stream);

/* Mean (nx) and covariance (row-major nx x nx) of the current density, FP64: the
 * first two moments of the point-mass density (the moment relations of Sec. II.A;
 * the estimates whose errors Sec. VI reports as RMSE and ASTD), as node sums with
 * the grid's integration weights (point masses on a Fourier grid, Clenshaw-Curtis
 * weights on a Chebyshev grid).
 * Synchronises `stream`.  Returns the status word collected since the last
 * synchronising call (PMF_E_DEGENERATE and/or PMF_W_BOUNDARY bits) and clears it. */
pmf_status pmf_moments(pmf_filter* f, double* mean, double* cov, void* stream);

/* Synchronise `stream` and return / clear the status word as pmf_moments does. */
pmf_status pmf_sync_status(pmf_filter* f, void* stream);

/* Substeps the last pmf_predict used (synchronises the null stream). */
pmf_status pmf_last_substeps(pmf_filter* f, int* l);

/* Copy grid + density to a host image.  If host_buf is NULL, only *bytes is set.
 * Synchronous (device synchronise). */
pmf_status pmf_get_state(pmf_filter* f, void* host_buf, size_t* bytes);

/* Replace grid + density from a host image written by pmf_get_state of a filter
 * with the same nx, grid kind, N and precision.  Synchronous. */
pmf_status pmf_set_state(pmf_filter* f, const void* host_buf, size_t bytes);

/* One predict(T) + update(z) cycle for n >= 1 filters in one fused launch
 * (Fourier grids, FP32 densities; nx = 2 with N0 x N1, N0 and N1 each in 32, 48,
 * 64, 96, 128 (square or rectangular); nx = 1 with N in 32, 48, 64, 96, 128, 192,
 * 256; other filters, n < 1 and NULL arguments are rejected with PMF_E_INVALID
 * before anything runs).  RK4 and Euler filters take at most 64 substeps in the
 * fused form: one whose clamp asks for more at run time is left as it was by
 * the cycle (grid, time, density up to FP32 rounding) with PMF_E_INVALID in its
 * status word, for the caller to step it through pmf_predict / pmf_update.
 * z: n * nz_max doubles, row f holds filter f's measurement (nz_max = largest nz);
 * copied into pinned staging before the call returns (the caller may reuse it).
 * loglik: NULL or n doubles written by an asynchronous copy (as pmf_update).
 * Each filter may appear once (a repeated filter is rejected).  The launch
 * set-up (grouping, device tables) is cached per (filter set, T, stream); a
 * step is then two kernel launches (per-filter planning, fused cycle) and z
 * goes through one of several mapped staging slots, so up to four steps can be
 * in flight before the call blocks.  Results equal n separate pmf_predict +
 * pmf_update calls up to FP32 rounding of the likelihood shift.  Async. */
pmf_status pmf_batch_step(pmf_ctx* ctx, pmf_filter* const* filters, int n, double T,
                          const double* z, double* loglik, void* stream);

/* K cycles predict(T) + update(z_k) of n filters back to back, for measurements
 * known ahead (replays, offline passes, benchmarks): the same filters, results
 * and rules as K calls of pmf_batch_step (bit for bit).  z: K rows of n * nz_max
 * doubles (row k: step k, filter order as `filters`); loglik: NULL or K * n
 * doubles (row k: step k).  1 <= K <= 256.  The K steps' launches (planning and
 * fused kernel per step) are captured into one HIP graph per filter set, T and K,
 * cached with the batch set-up, and replayed on a private stream after one copy
 * of all K rows of z.  Synchronous: waits for the caller's `stream` first, and
 * returns when the K steps have completed and loglik is written. */
pmf_status pmf_batch_run(pmf_ctx* ctx, pmf_filter* const* filters, int n, double T, int K,
                         const double* z, double* loglik, void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): pmf_batch_step without
 * any allocation.  Same arguments, filters and results as pmf_batch_step, at most
 * 4096 filters (more -> PMF_E_INVALID before anything runs).  The per-step
 * records (items, groups, plans, staged z, log-likelihoods; under
 * 2 MiB) live in a file-scope device array that each GPU holds until the process
 * ends; the per-filter constants live in the filter (allocated by pmf_create).
 * No hipMalloc/hipFree or other allocating call is made.  Synchronous: returns
 * once the step has completed on `stream` and loglik (NULL ok, n doubles, any
 * host memory) is written.  Every call on one GPU uses that GPU's one array:
 * calls from threads of one process are serialised by a lock; calls that
 * overlap on one GPU by other means race.  Nothing is cached between calls. */
pmf_status pmf_batch_step_noalloc(pmf_ctx* ctx, pmf_filter* const* filters, int n, double T,
                                  const double* z, double* loglik, void* stream);

/* Kernel timing of batched steps: with enable != 0, every later pmf_batch_step
 * also records HIP events on its stream right before and after the fused
 * kernel.
 * pmf_batch_kernel_time synchronises the context's last batch stream and
 * returns the summed event time (ms) of the fused kernel and the number of
 * launches since the previous call, then clears them.  Diagnostic. */
pmf_status pmf_batch_profile(pmf_ctx* ctx, int enable);
pmf_status pmf_batch_kernel_time(pmf_ctx* ctx, double* total_ms, int* launches);

/* Schedule autotuning of the fused batched step.  The fused kernel carries
 * compile-time schedule variants per 2-D grid size N x N (N in 32, 48, 64, 96,
 * 128): 0 the default; bit 0 (1) half the filters per workgroup (offered where
 * more than one fits); bit 1 (2) the radix passes of the column transforms in
 * reverse order (offered where that changes the radix plan).  All variants
 * compute the same cycle and differ in rounding only (the radix order; the rows
 * each thread sums in the FP64 reductions, which follow the filters per
 * workgroup).  1-D sizes have the default only.  A context starts with variant
 * 0 everywhere.
 *
 * pmf_autotune: tunes the variants for a mix of 2-D sizes.  counts[0..4] (NULL:
 * 1024 each) are the numbers of filters of size 32, 48, 64, 96 and 128 per axis
 * in the batches the caller will step (0..65536 each, at least one filter in
 * all).  The tuner creates that many synthetic fusable filters (a sheared
 * stable drift, a linear measurement of both components, exact integrator,
 * FP32) and times `steps` (1..1000) batched steps of the whole mix with HIP
 * events around the fused kernel, after two untimed steps.  Starting from the
 * defaults it takes the sizes present, largest first, and for each times every
 * offered variant on the mix (three rounds, each variant's fastest mean kept),
 * keeping the fastest if it beats the default by at least 1 % (one pass of
 * coordinate descent).  The choice stays in the context: later pmf_batch_step,
 * pmf_batch_step_noalloc and server batches of the context use it.
 * cache_path: NULL, or a JSON file.  If it exists and its "key" matches this
 * device (architecture, compute units), HIP runtime version, library build and
 * mix, its "schedules" are taken and nothing is timed; else the mix is timed
 * and the file is written (replaced).  report: NULL, or a buffer of report_len
 * bytes for a text summary (one line per size).  Synchronous; creates and
 * destroys its synthetic filters, drops the context's cached batch set-up and
 * clears the pmf_batch_profile timings; on failure the context's schedules are
 * left as they were.  Not to be called while other threads use the context. */
pmf_status pmf_autotune(pmf_ctx* ctx, const int* counts, int steps, const char* cache_path, char* report,
                        size_t report_len);

/* Schedule variant used for nx-D grids of N points per axis (nx = 1 or 2, a size
 * pmf_batch_step accepts; else PMF_E_INVALID).  pmf_set_schedule accepts only a
 * variant offered for that size (see pmf_autotune) and drops the context's
 * cached batch set-up when the variant changes. */
pmf_status pmf_get_schedule(pmf_ctx* ctx, int nx, int N, int* variant);
pmf_status pmf_set_schedule(pmf_ctx* ctx, int nx, int N, int variant);

/* ------------------------------------------------------------------ serving
 * Many independent tracks (one filter each) fed by an asynchronous stream of
 * requests, served by continuous batching: a native worker thread puts the next
 * op of every idle track with queued ops on the device as soon as the track is
 * free, without waiting for the work already running (finished work is found by
 * event queries).  A track whose FIFO starts with predict(T) followed by update(z)
 * and that pmf_batch_step accepts (Fourier, FP32, nx <= 2, the sizes listed
 * there) runs that pair as one fused cycle, batched with the other such tracks
 * taken in the same pass that have the same T (up to 4 fused batches on the
 * device at once); every other op runs through pmf_predict / pmf_update on the
 * least loaded of 4 HIP streams, concurrently with the fused batches, a predict
 * and the update queued after it as one run (back to back on that stream).  One
 * op, fused pair or run of a track is on the device at a time, so a track's ops
 * run in submission
 * order; results equal the direct calls on the same filter (fused pairs: bit for
 * bit equal to pmf_batch_step of the filter alone).  Admission: a track that
 * does not fit the server's device-memory budget waits (its ops are queued)
 * until pmf_server_remove_track frees memory; waiting tracks are admitted in the
 * order they were added.  The server owns its tracks' filters.  A server's
 * functions may be called from any thread; the filters of its tracks must not be
 * used directly while ops of theirs are queued or running. */
typedef struct pmf_server pmf_server;

typedef enum { PMF_OP_PREDICT = 0, PMF_OP_UPDATE = 1 } pmf_op;

typedef struct {
    long long tag;        /* the caller's tag of the request */
    int track;
    int op;               /* pmf_op */
    int status;           /* PMF_OK, or PMF_E_DEGENERATE for a rejected update */
    int fused;            /* 1 if the op ran in a fused batched cycle */
    double loglik;        /* update: log p(z_k | z^{k-1}) (NaN if rejected); predict: 0 */
    double latency_us;    /* submission to completion, host clock */
} pmf_completion;

typedef struct {
    size_t budget_bytes, used_bytes;   /* device bytes of the admitted tracks' filters */
    int tracks;                        /* admitted tracks */
    int waiting_tracks;                /* tracks waiting for memory */
    long long submitted, completed;
    long long rounds;                  /* worker passes that put work on the device */
    long long fused_ops, single_ops;
    long long admitted_late;           /* tracks admitted after waiting */
} pmf_server_stats;

/* Server on ctx with a device-memory budget for its tracks (admission control)
 * and at most max_tracks live tracks. */
pmf_status pmf_server_create(pmf_ctx* ctx, size_t budget_bytes, int max_tracks, pmf_server** out);

/* Blocks until every submitted op has completed, then frees the tracks. */
void pmf_server_destroy(pmf_server* s);

/* New track (the model is validated as pmf_create does).  If its device bytes
 * fit the budget and no earlier track is waiting, its filter is created now;
 * otherwise the track waits for memory: *track is set and ops may be submitted
 * to it, and it is created (and its ops run) once removals free enough memory.
 * PMF_E_NOMEM, with nothing kept, when max_tracks tracks are live or its device
 * bytes exceed the whole budget.  A waiting track whose creation then fails has
 * its queued ops completed with that error. */
pmf_status pmf_server_add_track(pmf_server* s, const pmf_model* model, const pmf_prior* prior, int* track);

/* Removes an idle (or waiting) track (PMF_E_BUSY while it has queued or running
 * ops), then admits waiting tracks that now fit. */
pmf_status pmf_server_remove_track(pmf_server* s, int track);

/* Queue one op: PMF_OP_PREDICT over T (z unused) or PMF_OP_UPDATE with z[0..nz)
 * (T unused).  Copies z; returns at once. */
pmf_status pmf_server_submit(pmf_server* s, int track, int op, double T, const double* z, long long tag);

/* Queue predict(T) then update(z) as one unit (no op of another submission can
 * come between them), tagged tag and tag + 1.  Returns at once. */
pmf_status pmf_server_submit_cycle(pmf_server* s, int track, double T, const double* z, long long tag);

/* Move up to cap completions (oldest first) into out; *n = how many. */
pmf_status pmf_server_poll(pmf_server* s, pmf_completion* out, int cap, int* n);

/* Block until every op submitted so far has completed (ops of tracks still
 * waiting for memory excepted). */
pmf_status pmf_server_drain(pmf_server* s);

pmf_status pmf_server_stats_get(pmf_server* s, pmf_server_stats* out);

/* The filter of an idle track, for pmf_get_state / pmf_moments (NULL if the
 * track does not exist or waits for memory). */
pmf_filter* pmf_server_filter(pmf_server* s, int track);

/* Device pointer of the density (for zero-copy inspection in tests); valid until
 * the next call on the filter.  Returns NULL on error. */
void* pmf_density_ptr(pmf_filter* f);

/* Wait for all work enqueued on `stream` (NULL = null stream). */
pmf_status pmf_stream_sync(void* stream);

const char* pmf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PMF_H */
