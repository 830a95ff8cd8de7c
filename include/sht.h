/*
 * sht.h -- C ABI of the MI355X (gfx950) scalar spherical harmonic synthesis
 * library, after D. S. Seljebotn, "Wavemoth -- Fast spherical harmonic
 * transforms by butterfly matrix compression" (arXiv:1110.4874).
 *
 * Problem (Sec. 1 Eq. 1, Sec. 2.1 Eq. 2): given coefficients a_lm of a real
 * field (a_{l,-m} = (-1)^m conj(a_lm), so only m >= 0 is stored), band limit
 * L, evaluate f = sum_{l<=L} sum_{|m|<=l} a_lm Y_lm at the pixel centres of a
 * HEALPix grid with resolution nside (12 nside^2 pixels on 4 nside - 1
 * iso-latitude rings, RING order).  The transform is computed as in Sec. 2.3
 * and 2.4: per-m Legendre phases q_m(z_k) on the rings (Eq. 12, using the
 * even/odd ring symmetry of Eqs. 13-14), then one real backward FFT per ring
 * after phase shift and wrap (Eqs. 8-11).
 *
 * Conventions shared by every entry point
 *   - All functions are extern "C", never throw and never abort.  They
 *     return an sht_status (0 on success); sht_last_error() gives a
 *     thread-local message for the last failure on the calling thread.
 *   - Array arguments named alm, map, q, workspace are DEVICE pointers
 *     (memory of the GPU the plan was built on).  Host pointers are rejected
 *     with SHT_EINVAL before anything is launched.  The caller owns them.
 *   - alm layout: complex128 (re, im) pairs, m-major with l ascending inside
 *     each m and the nmaps maps interleaved (Sec. A.3):
 *         alm[2*((off(m) + l - m)*nmaps + b) + {0,1}],  off(m) = m(2L+3-m)/2.
 *     Im a_l0 is ignored by synthesis (real field).
 *   - map layout: float64, stacked maps, RING order: map[b*Npix + p].
 *     (The paper interleaves output maps; stacked maps are kept here so that
 *     each ring is one contiguous, coalesced run per map.)
 *   - q layout (Legendre phase): complex128, ring-major then m then map:
 *         q[2*((k*(L+1) + m)*nmaps + b) + {0,1}],  ring k = 0..4nside-2
 *     (k = 0 is the northernmost ring).
 *   - Work is enqueued on the stream given in sht_exec_opts (NULL = the
 *     default stream) and is asynchronous with respect to the host.  Errors
 *     raised by the device are reported by a later call.
 */
#ifndef SHT_H
#define SHT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sht_plan_s sht_plan_t;

typedef enum {
    SHT_OK = 0,
    SHT_EINVAL = -1,       /* bad argument (range, null, host pointer, layout) */
    SHT_ENOMEM = -2,       /* host or device allocation failed, or workspace too small */
    SHT_EDEVICE = -3,      /* HIP runtime error, or a host-only plan used for compute */
    SHT_ECORRUPT = -4,     /* plan file failed its integrity checks (truncated,
                              altered, or not a plan file) */
    SHT_EUNSUPPORTED = -5, /* valid request outside what the library supports */
    SHT_EIO = -6           /* a plan file could not be opened, read or written */
} sht_status;

enum {
    SHT_PATH_AUTO = 0,      /* butterfly when the plan has it (eps > 0), else brute force */
    SHT_PATH_BRUTE = 1,     /* recurrence over every (l, ring) above the cutoff (App. A.2) */
    SHT_PATH_BUTTERFLY = 2, /* compressed operator of Sec. 3.2; needs an eps > 0 plan */
    SHT_PATH_INTERP = 3     /* Legendre phase at the roots of P~_N^m, then exact
                               interpolation to the rings (Sec. 3.3 Eq. 23); needs a
                               plan built with opts.interp = 1; synthesis only */
};

/* Arithmetic of the butterfly level products (sht_exec_opts.precision).
 * The residual recurrence, the fold and the ring FFT stay FP64. */
enum {
    SHT_PREC_FP64 = 0,
    SHT_PREC_FP32 = 1       /* FP32 interpolation matrices and vectors with FP32
                               accumulation (plan built with store_fp32) */
};

/* Stages of a transform, for sht_exec_opts.stage_events. */
enum {
    SHT_STAGE_LEGENDRE = 0,      /* synthesis: Legendre phase q_m(z_k) */
    SHT_STAGE_RING = 1,          /* synthesis: phase shift, wrap, ring FFT */
    SHT_STAGE_RING_ADJ = 2,      /* adjoint: ring FFT, unwrap, weights */
    SHT_STAGE_LEGENDRE_ADJ = 3,  /* adjoint: transposed Legendre transform */
    SHT_STAGE_BF_RESIDUAL = 4,   /* butterfly synthesis: the residual launch */
    SHT_STAGE_BF_LEVELS = 5,     /* butterfly synthesis: the level launches (from the
                                    first to the last; recorded for one-batch plans) */
    SHT_NSTAGES = 6
};

/* Adjoint conventions (sht_exec_opts.adjoint_convention). */
enum {
    SHT_ADJ_TRANSPOSE = 0,  /* exact transpose of synthesis under the real inner
                               product sum_{l, m>=0} Re a Re g + Im a Im g:
                               weight 2 for m >= 1 (the gradient convention) */
    SHT_ADJ_DAGGER = 1      /* Y^dagger of Sec. 2.2 Eq. 7 restricted to m >= 0:
                               weight 1 for every m */
};

/* Options for building a plan.  Fill with sht_plan_opts_default() first. */
typedef struct sht_plan_opts {
    double cutoff;     /* Legendre values below this magnitude at the start of
                          each l-chain are skipped (App. A.2: 1e-30). */
    double dd_sin;     /* rings with sin(theta) below this threshold run the
                          recurrence in compensated double-double arithmetic;
                          < 0 selects the default 0.1 * L / 4095.  FP64
                          recurrences lose ~L eps / sin(theta) near the poles. */
    int nthreads;      /* host threads for plan construction; 0 = all cores */
    int rings_per_lane;/* rings each lane of the FP64 Legendre kernel owns:
                          1, 2 or 4 (0 = default 2); a tuning knob */
    int ring_threads;  /* workgroup size of the ring FFT kernel: 256, 512 or
                          1024 (0 = default 512); a tuning knob */
    int host_only;     /* 1: build host tables only (no device memory); such a
                          plan can be inspected but not executed */
    /* Butterfly compression (eps > 0 plans only; Sec. 3.2 and 3.4): */
    double rho;        /* cost of one stored interpolation entry relative to one
                          residual recurrence element when choosing the depth per
                          (m, parity); <= 0 selects the default 4 (measured on
                          MI355X for FP64 level products at 4 maps; FP32 level
                          products favour lower values) */
    int max_levels;    /* -1: depth from the rho cost model; 0: no compression;
                          > 0: exactly this many levels where the rows allow */
    int chunk;         /* column block width at level 1 (0 = default 64) */
    double id_safety;  /* IDs are taken at tolerance eps / id_safety (values
                          below 1 count as 1; 0 = default 4, which keeps both
                          the compressed synthesis and its transpose within
                          eps of the exact operator on the maps measured) */
    int store_fp32;    /* 1: also keep an FP32 copy of the interpolation
                          matrices for SHT_PREC_FP32 */
    int batch_mib;     /* > 0: run the orders in batches whose level vectors (at
                          4 maps, FP64) stay under this many MiB between
                          launches; 0 (default): all orders in one batch */
    int store_transpose; /* 1: also keep every interpolation matrix transposed
                          (and, with store_fp32, its FP32 copy), so that the
                          adjoint streams them with the same coalesced loads as
                          the synthesis; doubles the device memory of the
                          matrices.  0 (default): the adjoint reads the
                          synthesis copy with strided loads (same results up
                          to rounding, slower) */
    int interp;        /* 1: also build the interpolation form of Sec. 3.3: per
                          (m, parity) the roots of P~_N^m (N = m + t + 2 n_t,
                          n_t the chain length), the weights of Eq. 23 and
                          P~_N^m on every north ring (host, long double; about
                          a minute and 0.6 GB of device memory at L = 4095) */
} sht_plan_opts;

/* Options for one execution.  Fill with sht_exec_opts_default() first. */
typedef struct sht_exec_opts {
    int nmaps;                /* number of maps B >= 1 transformed together */
    int path;                 /* SHT_PATH_* */
    void *stream;             /* hipStream_t, NULL = default stream */
    void *workspace;          /* device scratch of >= sht_workspace_bytes(), or
                                 NULL to let the call allocate (stream ordered) */
    size_t workspace_bytes;
    int adjoint_convention;   /* SHT_ADJ_*, used by the adjoint only */
    int precision;            /* SHT_PREC_*, butterfly path only */
    void **stage_events;      /* NULL, or 2*SHT_NSTAGES hipEvent_t handles
                                 (entries may be NULL): events[2s] is recorded
                                 on the stream before stage s runs and
                                 events[2s+1] after it */
} sht_exec_opts;

/* Statistics of a plan. */
typedef struct sht_plan_info {
    int L, nside, nrings, n_dd_rings;
    double eps;
    long long n_step;         /* (l, ring) pairs of the north rings, both
                                 parities, whose Legendre value is at or above
                                 the cutoff: the brute-force work unit (each
                                 costs 5 flops of recurrence + 4 per map) */
    long long n_step_exec;    /* recurrence steps the kernel executes (chain
                                 starts rounded down to a chunk boundary) */
    long long n_step_dd;      /* executed steps in compensated ring blocks */
    long long n_step_lanes;   /* lane-steps the Legendre kernel issues (idle
                                 lanes of partially active waves included) */
    size_t device_bytes;      /* device memory held by the plan */
    double build_seconds;     /* wall time of sht_plan */
    /* butterfly (zero unless eps > 0) */
    int bf_built;
    long long bf_T_entries;   /* stored dense interpolation entries (FP64: 8 B each) */
    long long bf_res_elems;   /* residual recurrence elements (l, skeleton ring) */
    long long bf_nodes;       /* pair nodes over all (m, parity, level) */
    long long bf_units;       /* level output columns over all nodes */
    long long bf_res_lanes;   /* residual (leaf, skeleton ring) lanes */
    long long bf_res_exec;    /* lane-steps the residual kernel executes (>= bf_res_elems) */
    long long bf_depth_hist[11]; /* (m, parity) items per kept depth 0..10 */
    double bf_build_seconds;
    int bf_nbatch;            /* order batches per transform */
    long long bf_level_T[11];     /* dense entries of the pair nodes of level 0..10 */
    long long bf_level_units[11]; /* output columns of the pair nodes of level 0..10 */
    long long bf_level_nodes[11]; /* pair nodes of level 0..10 (each reads a 64-byte
                                     record and 2 n int16 column positions) */
    /* interpolation form (zero unless opts.interp) */
    int ip_built;
    long long ip_nodes;       /* node-phase points over all (m, parity): the
                                 Legendre-root nodes and the direct rings */
    long long ip_steps;       /* node chain steps above the cutoff (the node
                                 phase's work unit: 5 flops + 4 per map) */
    long long ip_exec;        /* lane-steps the node kernel executes */
    double ip_build_seconds;
    long long ip_direct;      /* (order, parity, ring) values evaluated at the
                                 ring itself: rings closer to a node than the
                                 nodes' long-double precision allows for */
    int pol_rings;            /* north rings (each with its south mirror) where the
                                 polarized synthesis evaluates the spin-2
                                 functions directly */
} sht_plan_info_t;

void sht_plan_opts_default(sht_plan_opts *o);
void sht_exec_opts_default(sht_exec_opts *o);

/* Build a plan for band limit L >= 0 on a HEALPix grid of resolution
 * 1 <= nside <= 2048, on the current HIP device.  The plan holds the ring
 * geometry, the two-step recurrence coefficients of App. A.2 Eq. A2 and, per
 * (m, parity, ring), the first Legendre values above the cutoff (App. A.2):
 * everything the brute-force path needs.  eps > 0 additionally runs the FP64
 * butterfly precompute of Sec. 3.2 (interpolative decompositions at
 * tolerance eps, Eqs. 19-20, depth per (m, parity) from the cost model of
 * Sec. 3.4) on the host's cores and uploads the compressed operator; this
 * takes minutes at L = 4095 and tens of GB of device memory.
 * Returns NULL on failure (see sht_last_error).  The plan is immutable and
 * may be shared by threads; free it with sht_plan_free. */
sht_plan_t *sht_plan(int L, int nside, double eps);
sht_plan_t *sht_plan_ex(int L, int nside, double eps, const sht_plan_opts *opts);
void sht_plan_free(sht_plan_t *plan);
int sht_plan_info(const sht_plan_t *plan, sht_plan_info_t *out);

/* ---- plan files ---------------------------------------------------------
 * The precomputed data is built once and reused: the paper writes it to files
 * that its core loads, and excludes that load from every timing (Sec. 4.1,
 * Sec. 4.2; Table 1 lists the precompute cost that a file saves).
 *
 * sht_plan_save writes every host table of the plan (geometry, recurrence
 * coefficients, chain starts, ring FFT tables and, for eps > 0, the whole
 * compressed operator) to `path`: a versioned header holding L, nside, eps,
 * the options that shape the operator (cutoff, dd_sin, rho, max_levels, chunk,
 * id_safety, batch_mib, the tuning knobs and the store flags) and the
 * library's record layout, then the tables, with checksums over both.  The
 * file is written under a temporary name next to `path` and renamed into
 * place.  A device plan whose host copy of the interpolation data was
 * dropped after upload is read back from the device for the save (needs
 * that much host memory).  Returns SHT_EIO when the file cannot be written.
 *
 * sht_plan_load reads a file written by sht_plan_save and builds the plan on
 * the current HIP device, with the saved options; sht_plan_load_ex takes
 * host_only, store_fp32, store_transpose and nthreads (threads for the
 * checksum) from `opts` instead (NULL: as saved), so one file serves host-only
 * inspection, FP64-only and FP32 execution.  Both return NULL on failure;
 * sht_last_status() then gives SHT_ECORRUPT for a file that fails its
 * integrity checks (wrong magic, header or payload checksum mismatch, size
 * not matching the header, tables inconsistent with the geometry),
 * SHT_EUNSUPPORTED for a file written by a library with another version or
 * record layout, SHT_EIO when it cannot be opened, SHT_ENOMEM or SHT_EDEVICE
 * for allocation and upload failures.  The loaded plan computes exactly what
 * the saved one did. */
int sht_plan_save(const sht_plan_t *plan, const char *path);
sht_plan_t *sht_plan_load(const char *path);
sht_plan_t *sht_plan_load_ex(const char *path, const sht_plan_opts *opts);

/* Status of the last failed call on this thread (0 if none failed yet);
 * sht_last_error() gives its message.  Calls that return a pointer (plan
 * construction and loading) report their status here. */
int sht_last_status(void);

/* Device errors of asynchronous work: waits until the work queued on
 * `stream` (hipStream_t, NULL = default stream) on the plan's device has
 * finished, and returns SHT_EDEVICE with the HIP error text if the device
 * or the runtime reported an error for it, else SHT_OK.  Every transform
 * only enqueues work; this is the call that makes its failures visible
 * without a transform of its own. */
int sht_sync_status(const sht_plan_t *plan, void *stream);

/* Device scratch needed by one synthesis or adjoint with these options: the
 * Legendre phase buffer, nmaps * (L+1) * nrings complex values, plus on the
 * butterfly path the plan's vector workspace for up to 8 maps. */
size_t sht_workspace_bytes(const sht_plan_t *plan, const sht_exec_opts *x);

/* Synthesis f = Y a for one map (sht_synthesis) or x->nmaps maps. */
int sht_synthesis(const sht_plan_t *plan, const double *alm, double *map);
int sht_synthesis_ex(const sht_plan_t *plan, const sht_exec_opts *x,
                     const double *alm, double *map);

/* Polarized (spin-2) synthesis: Q and U maps from E- and B-mode
 * coefficients.  The Discussion of the paper notes that the transform of a
 * polarized map reduces to three scalar transforms (per mode), which also
 * amortises the streaming of the plan's data; here the three coefficient
 * sets of E and of B (the spin-2 functions written through the scalar
 * P~_l^m, P~_{l+-1}^m by two spin raisings) run as 6 x->nmaps maps through
 * one scalar Legendre phase of the chosen path, are combined per ring and
 * order into Q_m, U_m, and go through the scalar ring stage.  On the rings
 * nearest the poles (sin(theta) < 0.1 sqrt((L+1)/4096)), where the
 * combination would divide by sin^2(theta), the spin-2 functions are
 * evaluated by their own recurrence in double-double arithmetic instead.
 * Convention: a_{+-2,lm} = -(E_lm +- i B_lm), Q +- iU = sum a_{+-2,lm}
 * _{+-2}Y_lm with the spin-weighted harmonics of Goldberg et al. (1967)
 * (Condon-Shortley phase, as the scalar P~).
 * E, B: x->nmaps maps each in the alm layout of band limit L - 1 (a plan for
 * L serves polarized maps up to L - 1; Im of the m = 0 entries is ignored),
 * device memory, not modified.  QU: 2 x->nmaps maps of Npix doubles, Q of
 * map b at row b and U at row nmaps + b.  Workspace (x->workspace, or
 * allocated stream-ordered when NULL): sht_pol_workspace_bytes() of the
 * same options (0 for FP32 options).  FP64 only: SHT_EUNSUPPORTED for
 * x->precision = SHT_PREC_FP32, since the combination's division by
 * sin^2(theta) would magnify the FP32 products' error.  Returns SHT_EINVAL
 * for L < 1 or bad pointers and the errors of sht_synthesis_ex. */
size_t sht_pol_workspace_bytes(const sht_plan_t *plan, const sht_exec_opts *x);
int sht_pol_synthesis(const sht_plan_t *plan, const sht_exec_opts *x, const double *E, const double *B,
                      double *QU);

/* Synthesis that allocates nothing, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  Same arguments, kernels and results as
 * sht_synthesis_ex, except that the workspace is a fixed array of
 * sht_noalloc_scratch_bytes() (64 MiB) that the library holds on every GPU it
 * runs on until the process ends (x->workspace is ignored).  The caller
 * still passes the input and output buffers.  Returns SHT_ENOMEM, before
 * anything is launched, when sht_workspace_bytes() of the same options
 * exceeds that size (e.g. L = 1023 at nside = 512 fits one map, L = 511 at
 * nside = 256 seven).  Calls on one GPU share the array: calls that overlap
 * in time on one GPU (other streams, other threads) race and must not be
 * made; calls ordered on one stream are safe.  No part of the array needs
 * to start at zero. */
size_t sht_noalloc_scratch_bytes(void);
int sht_synthesis_noalloc(const sht_plan_t *plan, const sht_exec_opts *x,
                          const double *alm, double *map);

/* Adjoint g = A^T y of synthesis (Sec. 2.2: the operator the Wiener filter of
 * Eq. 7 needs; the paper builds synthesis only).  With the default
 * convention SHT_ADJ_TRANSPOSE,
 *     g_lm = w_m sum_k P~_l^m(z_k) sum_j y_kj e^{-i m phi_kj},
 * w_0 = 1 (Im g_l0 = 0), w_m = 2 for m >= 1, so that
 * <synthesis(a), y> = sum Re a Re g + Im a Im g for real-field a.
 * map: x->nmaps stacked maps (input); alm: output in the alm layout.
 * The Legendre functions are recomputed (nothing is kept from synthesis).
 * x->path picks the Legendre part as for synthesis: the brute-force
 * recurrence (deterministic), or on an eps > 0 plan the transposed butterfly
 * (Sec. 3.2 factorization applied backwards; x->precision FP32 runs its
 * interpolation products on FP32 matrix cores), which is the exact transpose
 * of that plan's compressed synthesis.  The butterfly adjoint adds the
 * residual rows into alm with device atomics, so its last bits may differ
 * between runs.  The workspace is sht_workspace_bytes() of the same options. */
int sht_adjoint(const sht_plan_t *plan, const double *map, double *alm);
int sht_adjoint_ex(const sht_plan_t *plan, const sht_exec_opts *x, const double *map,
                   double *alm);

/* Spherical-harmonic analysis by the quadrature rule of Sec. 2.2
 * (a_lm = sum_j w_j f_j Y*_lm(theta_j, phi_j)) with the HEALPix grid's equal
 * pixel weight w = 4 pi / Npix, followed by `iterations` >= 0 Jacobi steps
 *     a <- a + w Y^dagger (f - Y a)
 * that correct the grid's non-orthogonality (a band-limited map with
 * L <= 2 nside - 1 is recovered to rounding in a dozen steps).  Y^dagger is
 * the SHT_ADJ_DAGGER adjoint (m >= 0, Im a_l0 = 0).  map: x->nmaps stacked
 * maps (input, not modified); alm: output in the alm layout.  Every step
 * runs the synthesis and adjoint kernels of x->path and x->precision, plus
 * element-wise update kernels.  x->adjoint_convention is ignored.  The
 * workspace is sht_analysis_workspace_bytes() of the same options (the
 * synthesis workspace plus one residual map set and one alm set); without
 * one the call allocates it on x->stream.  Returns SHT_EINVAL for
 * iterations < 0 or iterations > 1000. */
size_t sht_analysis_workspace_bytes(const sht_plan_t *plan, const sht_exec_opts *x);
int sht_analysis_ex(const sht_plan_t *plan, const sht_exec_opts *x, const double *map, double *alm,
                    int iterations);

/* ---- batches of requests ---------------------------------------------
 * Many independent syntheses (possibly of different L, nside and map
 * counts) in one call: the many-transform regime of Sec. 3.4.  Requests run
 * longest first on the least-loaded of nstreams internal default-priority
 * streams that fork from and join into o->stream through events; the call
 * allocates nothing (the workspace is required) and only enqueues, so a
 * whole batch can be captured into one HIP graph on o->stream.  Results are
 * identical to sht_synthesis_ex of each request.  Requests must not share
 * output buffers; all plans must live on one device.
 * Callers: many-map pipelines and serving loops. */
typedef struct sht_request {
    const sht_plan_t *plan;
    int nmaps;
    const double *alm;        /* device, the plan's alm layout for nmaps maps */
    double *map;              /* device, nmaps * Npix doubles */
} sht_request;

typedef struct sht_batch_opts {
    void *stream;             /* hipStream_t the batch is ordered on */
    int nstreams;             /* internal streams used, 1..8 (default 4) */
    int path;                 /* SHT_PATH_* for every request */
    int precision;            /* SHT_PREC_* for every request */
    void *workspace;          /* device scratch of >= sht_batch_workspace_bytes()
                                 (sht_queue_workspace_bytes() for sht_batch_create) */
    size_t workspace_bytes;
    int rings_per_lane;       /* work-queue batches: rings per lane of the Legendre
                                 waves, 1, 2 or 4 (0 = 2); a tuning knob */
    int ring_threads;         /* work-queue batches: ring FFT workgroup size, 256,
                                 512 or 1024 (0 = 512); a tuning knob */
} sht_batch_opts;

void sht_batch_opts_default(sht_batch_opts *o);
size_t sht_batch_workspace_bytes(const sht_request *reqs, int n, const sht_batch_opts *o);
int sht_batch_execute(const sht_request *reqs, int n, const sht_batch_opts *o);

/* ---- work-queue batches ----------------------------------------------
 * The same many-request synthesis prepared once and replayed with a fixed,
 * small number of launches, for serving loops and graph capture
 * (many-transform regime of Sec. 3.4).  sht_batch_create splits the
 * brute-force Legendre phase of every request into work items (pass of up
 * to 4 maps, order m, block of ring groups), sorts them longest first by
 * their chain steps and uploads them with their argument blocks; it
 * allocates those tables (freed by sht_batch_free) and fixes every address
 * it was given.  sht_batch_run enqueues on `stream` (hipStream_t, NULL =
 * default) one persistent Legendre launch whose waves take items from a
 * device counter until none are left, then one ring-FFT launch per ring
 * size class covering every request (sht_batch_stats reports the item and
 * launch counts and the waves of the persistent launch); it allocates nothing and waits for nothing, so a run can
 * be captured into a HIP graph and replayed.  Results equal
 * sht_synthesis_ex of each request on the brute-force path bit for bit.
 * o->path must be SHT_PATH_BRUTE (others: SHT_EUNSUPPORTED); o->workspace
 * must hold sht_queue_workspace_bytes() (every request's Legendre phase),
 * and it, the alm inputs and the map outputs must stay valid, and must not
 * be used by other work while a run is in flight, for the batch's life.
 * Runs of one batch that overlap in time race.  o->nstreams is ignored.
 * Callers: serving loops and pipelines that replay a fixed set of
 * transforms. */
typedef struct sht_batch_s sht_batch_t;
size_t sht_queue_workspace_bytes(const sht_request *reqs, int n, const sht_batch_opts *o);
sht_batch_t *sht_batch_create(const sht_request *reqs, int n, const sht_batch_opts *o);
int sht_batch_run(const sht_batch_t *batch, void *stream);
int sht_batch_stats(const sht_batch_t *batch, long long *items, int *launches, int *waves);
void sht_batch_free(sht_batch_t *batch);

const char *sht_last_error(void);

/* ---- private test API (the paper's unit-test entry points, Sec. 4.1) ---- */

/* Legendre phase only: q_m(z_k) for every m and ring (Sec. 2.4 Eq. 12),
 * written to q in the layout above. */
int sht_debug_legendre_phase(const sht_plan_t *plan, const sht_exec_opts *x,
                             const double *alm, double *q);

/* Ring stage only: phase shift, wrap and real backward FFT per ring
 * (Sec. 2.3 Eqs. 8-11) from a given q to the map. */
int sht_debug_ring_synthesis(const sht_plan_t *plan, const sht_exec_opts *x,
                             const double *q, double *map);

/* Host-side tables (valid also for host_only plans), copied to host memory:
 *   coef: for order m, (L - m + 1) entries of (beta_l, alpha_l*beta_l,
 *         gamma_l) of the two-step recurrence
 *         P_{l+2} = (z^2 + alpha_l) beta_l P_l + gamma_l P_{l-2}
 *         (App. A.2 Eq. A2), l = m..L, rounded to double.
 *   start: for order m, parity t and north ring k (0 <= k < 2 nside):
 *         *idx = first chain index i (l = m + t + 2i) held in the table,
 *         rounded down to the kernel's chunk (or >= chain length if the
 *         whole chain stays below the cutoff), vals[0..1] = P at i, i+1. */
/* Adjoint ring stage only: ybar_m(z_k) = w_m sum_j y_kj e^{-i m phi_kj} for
 * every m and ring, written in the q layout. */
int sht_debug_ring_analysis(const sht_plan_t *plan, const sht_exec_opts *x,
                            const double *map, double *ybar);

/* Adjoint Legendre stage only: g_lm = sum_k P~_l^m(z_k) ybar_m(z_k) from ybar
 * in the q layout to alm layout. */
int sht_debug_legendre_adjoint(const sht_plan_t *plan, const sht_exec_opts *x,
                               const double *ybar, double *alm);

int sht_debug_coef(const sht_plan_t *plan, int m, double *coef_out);

/* Interpolative decomposition of Sec. 3.1 on the host, as the butterfly
 * precompute takes it: A is r x c column-major (not modified), tol the
 * relative tolerance.  Writes the rank to *k, the column order to piv[c]
 * (piv[0..k) are the skeleton columns) and T (k x (c-k), row-major) with
 * A[:, piv[k+j]] ~= sum_s A[:, piv[s]] T[s][j]; T must hold c*c doubles. */
int sht_debug_interp_decomp(const double *A, int r, int c, double tol, int *k, int *piv, double *T);

/* Host evaluation of q^t_m(z_k) = sum_i Lambda[i][k] x_i over the north
 * rings from the plan's compressed records (residual recurrence + levels),
 * for x of length n_t = (L - m - t)/2 + 1 (real).  y: n_north doubles.
 * Needs an eps > 0 plan whose interpolation data is still on the host
 * (plans under 256 MiB of it). */
int sht_debug_butterfly_apply(const sht_plan_t *plan, int m, int t, const double *x, double *y);

/* Host evaluation of q^t_m(z_k) over the north rings through the plan's
 * interpolation form (node chains from the stored starts, then Eq. 23), for
 * x of length n_t = (L - m - t)/2 + 1 (real).  y: n_north doubles.  Needs a
 * plan built with opts.interp = 1 (host_only plans included). */
int sht_debug_interp_apply(const sht_plan_t *plan, int m, int t, const double *x, double *y);
/* Test entry point: _s lambda_lm (s = +-2) at polar ring k (0 <= k <
 * pol_rings, ring k+1 of the RING scheme) by the host form of the polarized
 * synthesis' polar recurrence; out[l - m], l = m .. L - 1. */
int sht_debug_pol_column(const sht_plan_t *plan, int m, int s, int k, double *out);

/* Depth kept for (m, t) of an eps > 0 plan, or -1. */
int sht_debug_butterfly_depth(const sht_plan_t *plan, int m, int t);
int sht_debug_start(const sht_plan_t *plan, int m, int t, int k, int *idx,
                    double *vals);

#ifdef __cplusplus
}
#endif
#endif /* SHT_H */
