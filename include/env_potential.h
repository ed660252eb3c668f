/*
 * env_potential.h -- C ABI of the MI355X (gfx950) environment-potential library.
 *
 * The library evaluates the electrostatic potential of a fixed QM/MM
 * environment at QMC electron positions (paper Sec. II.B, Eq.
 * ElectrostaticField, and the per-MC-step use of Sec. III):
 *
 *     V(r) = sum_A Z_A / |r - R_A|  -  sum_{mu,nu} P_{mu nu} [mu nu | r]
 *
 * with the environment electron density given by a density matrix P over
 * contracted Cartesian Gaussian basis functions.  The paper's field
 * U_ES(r) of Eq. ElectrostaticField is the potential energy of an electron,
 * U_ES = -V.  All quantities are in atomic units (bohr, hartree, e).
 *
 * The shape of the interface follows the paper's host/device split
 * (Sec. III): the read-only environment is uploaded once by
 * env_potential_create, and each evaluation moves only the electron
 * positions in and the potential out.  The nuclear and electronic parts are
 * summed on the device (the paper summed them on the host, Sec. III).
 *
 * Conventions
 *   Basis order      shells in array order; within a shell the Cartesian
 *                    components in x-major order: p = x, y, z;
 *                    d = xx, xy, xz, yy, yz, zz (six Cartesian d functions).
 *   Normalisation    coefs multiply normalised primitives; each contracted
 *                    Cartesian component is then rescaled to unit
 *                    self-overlap.
 *   Fragments        each nucleus carries a fragment id (>= 0, or -1 for
 *                    "none": those form one group of their own).  Density
 *                    elements between basis functions of different fragments
 *                    are accepted and accumulated in a separate cross group.
 *   Ownership        create deep-copies every input; the caller may free
 *                    them on return.  points/out of an evaluation belong to
 *                    the caller and must stay valid until the stream has
 *                    completed the evaluation.
 *   Streams          evaluation calls are asynchronous on the given HIP stream
 *                    (NULL = the default stream) and never synchronise the
 *                    host; a handle may be evaluated concurrently on several
 *                    streams.
 *   Errors           every call returns an env_status; no exception crosses
 *                    the ABI.  Arguments are validated before any device
 *                    work is queued.
 *   Device           evaluation runs on a gfx950 device; without one create
 *                    returns ENV_E_DEVICE unless ENV_BUILD_ONLY or
 *                    ENV_FORCE_CPU is set.  ENV_FORCE_CPU is the paper's switch
 *                    back to the CPU (Sec. I): the caller asks for it at create,
 *                    and the handle then evaluates on host threads from host
 *                    buffers.  A device handle never falls back to the CPU.
 */
#ifndef ENV_POTENTIAL_H
#define ENV_POTENTIAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct env_potential env_potential; /* opaque, immutable after create */

typedef enum {
    ENV_OK = 0,
    ENV_E_ARG = -1,         /* invalid argument (NULL, NaN, size, asymmetric P) */
    ENV_E_UNSUPPORTED = -2, /* valid but not supported (l > 2, option combination) */
    ENV_E_NOMEM = -3,       /* host or device allocation failed */
    ENV_E_DEVICE = -4,      /* no usable device, or a HIP call / launch failed */
    ENV_E_STATE = -5        /* handle cannot do this (e.g. built with ENV_BUILD_ONLY) */
} env_status;

typedef enum {
    ENV_PREC_FP64 = 0,  /* every step in FP64 */
    ENV_PREC_FP32C = 1  /* pair arithmetic in FP32, FP64 differences of coordinates,
                           FP32 tile sums promoted to FP64, FP64 nuclear term and
                           per-fragment nuclear-minus-electronic sums */
} env_precision;

/* Option flags */
#define ENV_BUILD_ONLY 0x1u       /* build the pair list on the host, touch no device;
                                     the handle supports info/export, not evaluation */
#define ENV_NEUTRALIZE 0x2u       /* rescale each fragment's diagonal density block so
                                     that its electron count tr(P_f S_f) equals the
                                     fragment's nuclear charge (needs a block-diagonal P) */
#define ENV_NO_SCREENING 0x4u     /* keep every primitive pair */
#define ENV_FORCE_CPU 0x10u       /* evaluate on the host instead of the device (paper
                                     Sec. I: the user can switch back to the CPU code):
                                     FP64 only (FP32C gives ENV_E_UNSUPPORTED), no
                                     device is touched, env_potential_eval takes host
                                     points/out and returns when they are written (the
                                     stream is ignored); every other evaluation call
                                     (field, batched, surrogate, density update,
                                     autotune) returns ENV_E_STATE.  Not combinable
                                     with ENV_BUILD_ONLY (ENV_E_ARG).  ENVPOT_THREADS
                                     sets the thread count (default: all cores). */
#define ENV_NO_MERGE 0x8u         /* evaluate every pair on its own: no same-centre
                                     clusters (results agree to rounding) */
#define ENV_HOST_PACK 0x20u       /* device handles: enumerate, screen, order and lay
                                     out the pairs on the host (the packer of
                                     ENV_BUILD_ONLY handles) instead of on the device;
                                     the records are the same bit for bit */

typedef struct {
    double xyz[3];     /* position, bohr */
    double Z;          /* nuclear charge (0 allowed: a basis-only centre) */
    int32_t fragment;  /* fragment id >= 0, or -1 */
    int32_t reserved;  /* must be 0 */
} env_nucleus;

typedef struct {
    int32_t atom;              /* index of the nucleus the shell sits on */
    int32_t l;                 /* angular momentum, 0..2 */
    int32_t nprim;             /* number of primitives, >= 1 */
    int32_t reserved;          /* must be 0 */
    const double* exponents;   /* nprim exponents, > 0 */
    const double* coefs;       /* nprim contraction coefficients */
} env_shell;

#define ENV_DENSITY_DENSE 0   /* values: nbf x nbf row-major */
#define ENV_DENSITY_CSR 1     /* row_ptr[nbf+1], col[nnz], values[nnz] */

typedef struct {
    int32_t nbf;              /* number of basis functions (must match the shells) */
    int32_t format;           /* ENV_DENSITY_DENSE or ENV_DENSITY_CSR */
    const double* values;
    const int64_t* row_ptr;   /* CSR only */
    const int32_t* col;       /* CSR only; both triangles of the symmetric P */
} env_density;

typedef struct {
    int32_t precision;        /* env_precision */
    int32_t device;           /* HIP device ordinal, -1 = current device */
    double screen_threshold;  /* primitive-pair screening threshold (default 1e-12) */
    uint32_t flags;           /* ENV_* option flags */
    int32_t reserved[3];      /* must be 0 */
} env_options;

typedef struct {
    int32_t nbf;
    int32_t n_nuclei;             /* nuclei with Z != 0 */
    int32_t n_groups;             /* fragment groups (incl. the cross group if used) */
    int32_t n_segments;
    int64_t n_pairs;              /* unique screened primitive shell pairs */
    int64_t n_pairs_by_L[5];      /* by L = l_I + l_J */
    int64_t n_pairs_unscreened;   /* unique primitive shell pairs in nonzero blocks */
    double electrons;             /* sum over pairs of the pair charge = tr(P S) after
                                     screening and neutralisation */
    double nuclear_charge;        /* sum of Z */
    double screened_bound;        /* sum over dropped pairs of |P|-weighted charge bound */
    int64_t device_bytes;         /* bytes held on the device by the handle */
    int32_t precision;
    int32_t built_on_device;      /* 0 with ENV_BUILD_ONLY or ENV_FORCE_CPU */
    int64_t n_clusters;           /* same-centre clusters (far fields merged per atom) */
    int64_t n_cluster_members;    /* pairs inside those clusters (counted in n_pairs too) */
    int32_t on_host;              /* 1 with ENV_FORCE_CPU: evaluation runs on host threads */
    int32_t pairs_built_on_device;/* 1 when the pairs were enumerated, screened, ordered
                                     and laid out on the device (see env_potential_create) */
} env_info;

/* Default options: FP32C, current device, threshold 1e-12, no flags. */
void env_options_default(env_options* opts);

/* Build the environment (paper Sec. II.B: nuclei {Z_beta, R_beta} plus the
 * electron density; Sec. III: uploaded once, read-only afterwards).
 * The host validates the inputs and parses the density into shell blocks;
 * for a device handle the device then enumerates every primitive pair of the
 * nonzero blocks, screens it, orders the kept pairs, forms the same-centre
 * clusters, writes the records and folds the density into them (ENV_HOST_PACK:
 * the host does the pairs and the layout, the device the fold; same records
 * bit for bit).  ENV_BUILD_ONLY and ENV_FORCE_CPU handles are built on the
 * host entirely.  Returns the handle in *out.
 * Errors: ENV_E_ARG (NULL pointers, n < 0, non-finite input, exponent <= 0,
 * atom index out of range, nbf mismatch, P not symmetric, ENV_FORCE_CPU with
 * ENV_BUILD_ONLY), ENV_E_UNSUPPORTED (l > 2; ENV_NEUTRALIZE with density
 * between fragments; ENV_FORCE_CPU with FP32C), ENV_E_NOMEM, ENV_E_DEVICE. */
env_status env_potential_create(const env_nucleus* nuclei, int32_t n_nuclei,
                                const env_shell* shells, int32_t n_shells,
                                const env_density* P, const env_options* opts,
                                env_potential** out);

/* V at n points (paper Sec. III: electron position in, potential out).
 * points: device pointer to n x 3 float64 (x, y, z of each point, contiguous);
 * out: device pointer to n float64.  stream: hipStream_t or NULL.
 * n = 0 is a no-op.  A point exactly on a nucleus gives +inf.
 * Calls of 32,768 points or more evaluate the points in a spatial (Morton)
 * order and write out in the caller's order (off while the stream is being
 * captured, or with ENVPOT_NO_SORT=1); the same call is bitwise repeatable.
 * A wave of points that is beyond the largest far-field radius of a pair
 * segment's bounding box runs that segment without the per-pair near test
 * (FP32C: with the coordinate differences formed from the wave's first
 * point, at most 3 FP32 ulps of |P - C|); ENVPOT_NO_FARBOX=1 at create turns
 * this off (then FP64 gives the same bits, FP32C agrees to rounding).
 * A handle created with ENV_FORCE_CPU takes host pointers instead, ignores
 * the stream and returns after writing out (FP64, the host threads of the
 * paper's switch back to the CPU).
 * Errors: ENV_E_ARG (NULL with n > 0, n < 0), ENV_E_STATE (ENV_BUILD_ONLY
 * handle), ENV_E_DEVICE (launch failure), ENV_E_NOMEM (workspace). */
env_status env_potential_eval(env_potential* h, const double* points, int64_t n,
                              double* out, void* stream);

/* Replace the environment's density matrix, keeping its geometry and basis
 * (an environment whose density changes from step to step, e.g. the
 * self-consistent fragment densities of FMO, Sec. II.B).  The pair list
 * (screening, order, same-centre clusters, splits) does not depend on the
 * density values, so the device refolds every pair's Hermite density and
 * far-field coefficients from the new P in place; with ENV_NEUTRALIZE the
 * per-fragment scaling is recomputed.  P: dense or CSR as at create, same
 * nbf; every nonzero block must be one that was nonzero at create (blocks
 * may become zero).  Synchronous on `stream`; no evaluation of h may run
 * meanwhile.  env_info.electrons is updated; screened_bound keeps the
 * create-time value.
 * Errors: ENV_E_ARG (nbf, format, non-finite or asymmetric P, a new
 * nonzero block), ENV_E_STATE (build-only handle), ENV_E_UNSUPPORTED (more
 * than 32767 primitives in a shell), ENV_E_DEVICE. */
env_status env_potential_update_density(env_potential* h, const env_density* P, void* stream);

/* The field E = -grad V together with V (an extension of the paper's
 * quantity, Sec. II.B, Eq. ElectrostaticField: the force on a unit positive
 * charge, whose negative is the electron's drift term).  For a pair the
 * gradient is the Hermite recursion one order further,
 *   d/dC [mu nu | C] = -(R_{t+1,u,v}, R_{t,u+1,v}, R_{t,u,v+1}) . D,
 * and for a nucleus Z (C - R_A) / |C - R_A|^3.
 * points: device n x 3 float64; out: device n x 4 float64 row-major
 * (V, E_x, E_y, E_z per point, hartree/e and hartree/(e bohr)).  Same
 * handle, precision and stream semantics as env_potential_eval; the
 * precision's far-field switch is applied one Boys order higher.  A point on
 * a nucleus gives non-finite values.  n = 0 is a no-op.
 * Errors: as env_potential_eval. */
env_status env_potential_eval_field(env_potential* h, const double* points, int64_t n,
                                    double* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same values
 * as env_potential_eval, with no device allocation and no Morton ordering
 * (the points are evaluated in the caller's order, as env_potential_eval
 * does below 32,768 points).  The split-pair partial sums go to a fixed
 * 64 MiB device array (2^23 float64) that the library holds on each device
 * it runs this call on until the process ends; the split factor is lowered
 * until split x n fits it.  Every call on one device shares that array, so
 * two calls whose executions overlap on one device (different streams, or
 * different handles on the same device) race and give wrong values: order
 * them on one stream or with events.  points, out, stream: as
 * env_potential_eval.  n = 0 is a no-op.
 * Errors: ENV_E_ARG (NULL with n > 0, n < 0, n above
 * env_potential_noalloc_max_points() = 8,388,608), ENV_E_STATE (host or
 * build-only handle), ENV_E_DEVICE (launch failure, symbol lookup). */
env_status env_potential_eval_noalloc(env_potential* h, const double* points, int64_t n,
                                      double* out, void* stream);
int64_t env_potential_noalloc_max_points(void);

/* Several independent evaluations in one persistent launch (convenience
 * form of the env_batch calls below): instance i evaluates handle hs[i] at
 * points[i] (n[i] x 3) into out[i] (n[i]).  All handles must be on the same
 * device with the same precision.  Unlike env_potential_eval this call
 * synchronises the stream before it returns (it owns temporary buffers).
 * Errors: as env_potential_eval; ENV_E_ARG for mixed devices/precisions. */
env_status env_potential_eval_batched(env_potential* const* hs, int32_t n_inst,
                                      const double* const* points, const int64_t* n,
                                      double* const* out, void* stream);

/* A reusable plan for repeated batched evaluation (many walkers and many
 * uneven QM/MM instances per QMC step; the paper's outlook of sharing one GPU
 * among several processes, Sec. I and Sec. V).  Work items (instance, point
 * block, pair range) are sorted by decreasing cost and drained by one
 * persistent kernel through a global work counter; split-pair partials are
 * reduced in fixed order, so a plan gives bitwise-identical results for the
 * same inputs on every call.  While the caller passes the same pointers and counts
 * on a non-NULL stream, env_batch_eval replays a captured HIP graph; a new
 * pointer set or count synchronises the stream once, uploads the new tables
 * and captures again.  The handles must outlive the plan. */
typedef struct env_batch env_batch;

typedef struct {
    int64_t n_items;          /* work items of the current shape */
    int32_t grid;             /* workgroups of the persistent launch */
    int32_t np;               /* points per lane of the current shape */
    int64_t launches;         /* direct launches */
    int64_t captures;         /* graph captures */
    int64_t graph_launches;   /* graph replays */
    int32_t granularity;      /* work items per workgroup's fair share of the work */
    int32_t reserved;
    int64_t sorted_points;    /* points of the instances evaluated in Morton order */
    int64_t sorts;            /* evaluations that sorted points */
    int64_t autotunes;        /* env_batch_autotune calls */
} env_batch_stats;

/* Errors: ENV_E_ARG (NULL, n_inst <= 0, mixed device/precision), ENV_E_STATE
 * (a build-only handle), ENV_E_NOMEM. */
env_status env_batch_create(env_potential* const* hs, int32_t n_inst, env_batch** out);

/* points[i]: device n[i] x 3 float64; out[i]: device n[i] float64.
 * Asynchronous on `stream` except when the pointers or counts changed.
 * Instances of 32,768 points or more are evaluated in Morton order (their
 * points are sorted into the plan's buffers before each launch; the values
 * are written back in the caller's order), as env_potential_eval does.
 * While `stream` is being captured by the caller, the launch is recorded
 * into the caller's graph without the sort (the plan's pointers and counts
 * must then be the ones of an earlier call: ENV_E_STATE otherwise). */
env_status env_batch_eval(env_batch* b, const double* const* points, const int64_t* n,
                          double* const* out, void* stream);

/* Pick the plan's launch shape for these pointers and counts: every pair of
 * points per lane (FP32C 2 or 4, FP64 1 or 2) and split granularity (4, 8 or
 * 16 work items per workgroup's fair share) is timed over two graph
 * replays; the fastest is kept for later calls with the same counts.
 * Writes out as env_batch_eval does.  Synchronous; stream must not be NULL.
 * Errors: as env_batch_eval, ENV_E_ARG for a NULL stream. */
env_status env_batch_autotune(env_batch* b, const double* const* points, const int64_t* n,
                              double* const* out, void* stream);

env_status env_batch_get_stats(const env_batch* b, env_batch_stats* stats);

void env_batch_destroy(env_batch* b);

/* ------------------------------------------------------------------------
 * One GPU shared by the processes of a node (the paper's outlook, Sec. I and
 * Sec. V: the GPU shared by the MPI processes running on the same node).
 * A server process owns the environments and the GPU; clients in other
 * processes (or threads) attach to it by name through POSIX shared memory
 * and submit evaluation requests with host buffers.  The server's worker
 * thread takes every request that is ready, evaluates them together in one
 * persistent batched launch (env_potential_eval_batched) and returns the
 * potentials.  Client calls make no HIP call: clients need no GPU context.
 * ------------------------------------------------------------------------ */
typedef struct env_server env_server;
typedef struct env_client env_client;

typedef struct {
    int64_t rounds;           /* batched launches */
    int64_t requests;         /* requests served */
    int64_t points;           /* points evaluated */
    int64_t errors;           /* requests answered with an error */
    double busy_seconds;      /* worker time spent serving rounds */
    int32_t clients;          /* slots currently attached */
    int32_t reserved;
} env_server_stats;

/* Serve the n_env handles (same device and precision; they must outlive the
 * server) under `name` ([^/]+, at most 200 characters; the segment is
 * /dev/shm/envpot.<name>).  n_slots: the most clients attached at once (one
 * request in flight each); max_points: the largest request; gather_us: how
 * long the worker waits after the first ready request before it takes all
 * ready requests (0: at once).  A segment of that name whose server process
 * is gone is replaced.
 * Errors: ENV_E_ARG, ENV_E_STATE (a build-only handle, or a live server of
 * that name), ENV_E_NOMEM, ENV_E_DEVICE. */
env_status env_server_create(env_potential* const* hs, int32_t n_env, const char* name, int32_t n_slots,
                             int64_t max_points, int32_t gather_us, env_server** out);

env_status env_server_get_stats(const env_server* s, env_server_stats* stats);

/* Stops the worker, answers requests still waiting with ENV_E_STATE and
 * removes the segment. */
void env_server_destroy(env_server* s);

/* Attach to the server `name` and claim a free slot.
 * Errors: ENV_E_ARG (bad name), ENV_E_STATE (no such live server, or every
 * slot taken), ENV_E_NOMEM. */
env_status env_client_attach(const char* name, env_client** out);

/* The server's environment count, request size limit and this client's slot. */
env_status env_client_info(const env_client* c, int32_t* n_env, int64_t* max_points, int32_t* slot);

/* V of environment `env` (index into the server's handles) at n host points
 * (n x 3 float64) into out (host, n float64); blocks until answered.
 * timeout_ms <= 0 waits as long as the server lives.  n = 0 is allowed.
 * Errors: ENV_E_ARG (bad env, n above max_points, NULL), ENV_E_STATE (the
 * server is gone, or the client is unusable after a time-out), ENV_E_DEVICE
 * (time-out, or a device error on the server), or the status the server's
 * evaluation returned. */
env_status env_client_eval(env_client* c, int32_t env, const double* points, int64_t n, double* out,
                           int32_t timeout_ms);

/* Release the slot (kept taken after a time-out) and unmap the segment. */
void env_client_detach(env_client* c);

/* Times the candidate launch shapes (points per lane, pair-split factor) of
 * h at the n device points `points` on `stream` (synchronous) and keeps the
 * fastest for evaluations of h at a point count within a factor 2 of n.
 * Must not run concurrently with other calls on the same handle.
 * Errors: ENV_E_ARG, ENV_E_STATE, ENV_E_NOMEM, ENV_E_DEVICE. */
env_status env_potential_autotune(env_potential* h, const double* points, int64_t n, void* stream);

/* Measurement support (not part of the method): with timing on, every later
 * env_potential_eval of h records a pair of HIP events on its stream around
 * the potential kernel alone (not the point ordering or the split sums), up
 * to 2048 launches; env_potential_kernel_timing(h, 1) also clears the list.
 * env_potential_kernel_times waits for the recorded events and writes the
 * kernel durations (ms) of the first min(cap, count) launches in call order;
 * *count receives the number recorded.  Not for concurrent evaluations of h.
 * Errors: ENV_E_ARG, ENV_E_STATE (host or build-only handle), ENV_E_DEVICE. */
env_status env_potential_kernel_timing(env_potential* h, int32_t on);
env_status env_potential_kernel_times(env_potential* h, float* ms, int32_t cap, int32_t* count);

/* Statistics of the built pair list. */
env_status env_potential_info(const env_potential* h, env_info* info);

/* Vector-ALU rates this device sustains, for roofline reports (measurement
 * support; not part of the method).  Runs three short kernels on `device`
 * (-1 = current): independent v_fma_f32 chains, v_fma_f64 chains and
 * v_rsq_f32 chains, eight per lane, 2048 iterations, 8192 x 256 threads.
 * Fills the achieved rates; blocks until done (about 10 ms).
 * Errors: ENV_E_ARG (NULL), ENV_E_DEVICE (no gfx950 device, launch failure),
 * ENV_E_NOMEM. */
typedef struct {
    double fp32_fma_tflops;   /* 2 flops per lane FMA */
    double fp64_fma_tflops;
    double rsq_f32_per_s;     /* lane reciprocal square roots per second */
    double ms[3];             /* kernel times: fma32, fma64, rsq32 */
} env_peak;
env_status env_peak_probe(int32_t device, env_peak* out);

/* Copy of the pair list for inspection (host buffers, any handle):
 * for each of the n_pairs pairs, in the library's internal order:
 *   L[k] (int32), group[k] (int32), center[3k..3k+2], exponent p[k] and the
 *   Hermite density D[35k .. 35k+ncomp(L)-1] (float64, scaled by
 *   (pi/p)^{3/2}, so that D[35k] is the pair's electron count), with the
 *   components t+u+v <= L ordered by t, then u, then v ascending.
 * Any output pointer may be NULL.  cap is the capacity in pairs; returns
 * ENV_E_ARG if cap < n_pairs. */
env_status env_potential_export_pairs(const env_potential* h, int64_t cap, int32_t* L,
                                      int32_t* group, double* center, double* p,
                                      double* D);

/* Copy of a device handle's record image for inspection (host buffers):
 * the records (rec_words 4-byte words: pair records, cluster records and the
 * clusters' member records of every fragment group) and the segment tables
 * of the split factors 1, 2, 4, ..., 256, concatenated (seg_words 4-byte
 * words, 8 per segment: L, count, first record word (int64), first and end
 * nucleus, flags, index of the unsplit segment it comes from).  Call with
 * NULL buffers to get the sizes; a buffer smaller than the size (cap in
 * words) gives ENV_E_ARG.  Waits for the device.  ENV_E_STATE for a host
 * handle. */
env_status env_potential_export_image(const env_potential* h, uint32_t* rec, int64_t rec_cap,
                                      int64_t* rec_words, uint32_t* segs, int64_t seg_cap,
                                      int64_t* seg_words);

/* ------------------------------------------------------------------------
 * Learned surrogate of V inside the QM region (not in the paper: an addition
 * of this library).  A coordinate MLP with Fourier-feature input,
 *     gamma(r) = [cos(2 pi B r), sin(2 pi B r)]   (B: 64 x 3, 1/bohr)
 *     4 hidden layers of 128 SiLU units, BF16 weights on the matrix cores with
 *     FP32 accumulation, an FP32 output layer 128 -> 1,
 *     V_hat(r) = poly(r/R) + sigma * y(r),
 * where poly is a least-squares polynomial baseline (monomials u_x^a u_y^b
 * u_z^c, a+b+c <= degree, ordered by total degree, then a descending, then b
 * descending).  It is trained on the GPU on samples of an exact handle; a
 * voxel gate validated against that handle decides, per point, whether the
 * network is used or the exact fallback handle is evaluated instead.
 *
 * Parameter vector (float32, 66,177 values): W1 (128 x 128, out x in), b1,
 * W2, b2, W3, b3, W4, b4, w_out (128), b_out.  Network inputs 0..63 are the
 * cosines, 64..127 the sines.
 * ------------------------------------------------------------------------ */
typedef struct env_surrogate env_surrogate;

typedef struct {
    int32_t n_freq;          /* must be 64 */
    int32_t hidden;          /* must be 128 */
    int32_t layers;          /* must be 4 */
    int32_t poly_degree;     /* 0..8 */
    double radius;           /* R: the region the surrogate covers is |r| <= R (bohr) */
    const double* B;         /* n_freq x 3 frequencies (1/bohr), host, copied */
    const float* params;     /* initial parameters (layout above), host, copied */
    const double* poly;      /* baseline coefficients (NULL allowed when poly_degree == 0) */
    double sigma;            /* output scale (<= 0 means 1) */
    int32_t reserved[4];
} env_surrogate_spec;

typedef struct {
    int64_t n_train;         /* samples uniform in the ball (default 2,000,000) */
    int32_t epochs;          /* default 20 */
    int32_t batch;           /* multiple of 32, default 8192 */
    double lr, lr_final;     /* Adam, cosine decay from lr to lr_final */
    uint64_t seed;           /* SplitMix64 seed of samples and shuffles */
    int32_t gate_grid;       /* G: voxels per axis over [-R, R]^3 (default 24) */
    int32_t gate_samples;    /* validation points per voxel (default 8) */
    double gate_tol;         /* a voxel passes if its max |V_hat - V| <= gate_tol (default 5e-6 Ha) */
    int64_t n_fit;           /* samples used for the baseline fit (default 131,072) */
    int32_t poly_degree;     /* baseline degree (default 6) */
    int32_t reserved[3];
} env_train_opts;

typedef struct {
    int64_t n_params;
    int32_t n_freq, hidden, layers, poly_degree;
    double radius, sigma, baseline_rms;
    int64_t train_steps;
    double final_loss;               /* last minibatch, normalised targets */
    double epoch_loss[64];           /* last minibatch of each epoch */
    double teacher_seconds, train_seconds, gate_seconds;
    int32_t gate_grid, reserved0;
    int64_t gate_voxels_in_ball, gate_voxels_pass;
    double gate_pass_volume_fraction; /* share of the ball's volume served by the network */
    double gate_max_err_passed;       /* largest validation error of a passing voxel */
    double gate_tol;
    int64_t last_eval_n, last_eval_fallback;
} env_surrogate_info;

void env_train_opts_default(env_train_opts* opts);

/* fallback: the exact handle evaluated for gated-out points (FP32C or FP64).
 * Errors: ENV_E_ARG, ENV_E_STATE (build-only fallback), ENV_E_UNSUPPORTED
 * (other sizes), ENV_E_NOMEM, ENV_E_DEVICE.  Synchronises the device once. */
env_status env_surrogate_create(env_potential* fallback, const env_surrogate_spec* spec,
                                env_surrogate** out);

/* Trains on opts->n_train points drawn uniformly in the ball with values from
 * `teacher`, fits the baseline, runs Adam, then validates the voxel gate
 * against `teacher`.  Synchronous.  Must not overlap other calls on s. */
env_status env_surrogate_train(env_surrogate* s, env_potential* teacher, const env_train_opts* opts,
                               void* stream);

/* Network + baseline at n device points (no gate): device out[n] float64. */
env_status env_surrogate_predict(env_surrogate* s, const double* points, int64_t n, double* out,
                                 void* stream);

/* Gated evaluation: points outside the ball or in a failed voxel are
 * evaluated by the exact fallback handle; used_fallback (device, n bytes,
 * may be NULL) receives 1 for them.  Asynchronous: the gated-out points are
 * compacted on the device and one persistent launch of the fallback's
 * kernel reads their count there and picks its split factor from it, so the
 * host never waits (the fallback values equal env_potential_eval's at the
 * compacted points to rounding: the split factor may differ and no Morton
 * ordering is applied).  With an exact part set (env_surrogate_set_near)
 * every other point gets network + baseline + the exact part's V.  Calls
 * on one surrogate must not overlap (they share its workspace).
 * ENV_E_STATE before training, after the fallback's density was updated
 * (env_potential_update_density), or when the exact part left the device. */
env_status env_surrogate_eval(env_surrogate* s, const double* points, int64_t n, double* out,
                              uint8_t* used_fallback, void* stream);

/* Split surrogate: the network stands in for the potential of part of the
 * environment only (the fragments far from the region, whose potential is
 * smooth there), and `near`, an exact handle of the remaining fragments (the
 * fragments of FMO, Sec. II.B, nearest the QM region), is evaluated at every
 * point and added.  Train such a surrogate with the far fragments' handle
 * as teacher; the fallback stays the handle of the whole environment, so a
 * gated-out point gets the whole environment's exact value.  near: a device
 * handle on the surrogate's device, or NULL to remove the exact part; it
 * must outlive its use.  Errors: ENV_E_ARG (s NULL), ENV_E_STATE (near not
 * a device handle of that device). */
env_status env_surrogate_set_near(env_surrogate* s, env_potential* near);

/* Diagnostic: loss mean((y - t)^2) and its gradient (host, 66,177 floats) for
 * the current parameters at n device points with device targets t (float32,
 * normalised).  Synchronous. */
env_status env_surrogate_loss_grad(env_surrogate* s, const double* points, const float* targets,
                                   int64_t n, float* grad_host, double* loss, void* stream);

/* Diagnostic: one forward and backward pass at n device points with device
 * targets t (float32, normalised), as env_surrogate_loss_grad, copying the
 * intermediate tensors to host buffers so that each layer can be checked on
 * its own.  Every pointer may be NULL (that tensor is skipped); row-major,
 * rows = points:
 *   H    (layers + 1) x n x 128   H_0 = the BF16 features, H_l = bf16(silu(Z_l)), as float
 *   Z    layers x n x 128         FP32 pre-activations Z_l = H_{l-1} bf16(W_l)^T + b_l
 *   y    n                        FP32 outputs H_4 . w_out + b_out
 *   dy   n                        dL/dy = 2 (y - t) / n as used by the backward pass
 *   dH   layers x n x 128         FP32 dL/dH_l, l = 1..4 (the input of each SiLU backward)
 *   dZ   layers x n x 128         bf16(dL/dH_l * silu'(Z_l)) fed to the weight products, as float
 *   grad 66,177                   the gradient in the parameter layout
 * Synchronous.  Errors: ENV_E_ARG, ENV_E_NOMEM, ENV_E_DEVICE. */
typedef struct {
    float* H;
    float* Z;
    float* y;
    float* dy;
    float* dH;
    float* dZ;
    float* grad;
    double loss;
} env_surrogate_trace;
env_status env_surrogate_trace_step(env_surrogate* s, const double* points, const float* targets, int64_t n,
                                    env_surrogate_trace* tr, void* stream);

/* Current parameters (host, 66,177 floats), baseline coefficients and sigma;
 * any pointer may be NULL. */
env_status env_surrogate_get_params(const env_surrogate* s, float* params, double* poly,
                                    double* sigma);

/* Statistics; last_eval_fallback is the gated-out count of the last
 * env_surrogate_eval, read after waiting for that call's stream. */
env_status env_surrogate_get_info(const env_surrogate* s, env_surrogate_info* info);

void env_surrogate_destroy(env_surrogate* s);

/* ------------------------------------------------------------------------
 * The paper's own form of the environment (Sec. II.B, Eq. ElectrostaticField;
 * Sec. III): nuclei plus the electron density given on M cells, each cell a
 * point charge q_m = rho(r_m) h^3 (electron count).  The library returns
 *     V(r) = sum_A Z_A / |r - R_A| - sum_m q_m / |r - r_m|,   U_ES = -V,
 * the same sign convention as env_potential_eval.
 * ------------------------------------------------------------------------ */
typedef struct env_cells env_cells;

/* Upload nuclei (fragment ids ignored; Z = 0 allowed) and cells (host, M x 4
 * row-major: x, y, z, q; bohr and electrons) once.  Options: precision
 * (ENV_PREC_FP64 or ENV_PREC_FP32C) and device; flags and the screening
 * threshold are ignored.  The inputs are copied.
 * Errors: ENV_E_ARG (NULL with a count > 0, negative counts, non-finite
 * values, M > 2^31 - 1), ENV_E_DEVICE (no gfx950 device), ENV_E_NOMEM. */
env_status env_cells_create(const env_nucleus* nuclei, int32_t n_nuclei, const double* cells,
                            int64_t n_cells, const env_options* options, env_cells** out);

/* V at n device points (n x 3 float64, row-major) into out (device, n
 * float64), asynchronous on `stream`.  Every point against every cell and
 * nucleus (a point on a nucleus gives +inf, a point on a cell a non-finite
 * value).  n = 0 is a no-op.
 * Errors: ENV_E_ARG, ENV_E_DEVICE, ENV_E_NOMEM (split partials). */
env_status env_cells_eval(env_cells* h, const double* points, int64_t n, double* out,
                          void* stream);

/* Single-point latency mode, one electron move at a time as in the paper's
 * QMC loop (Sec. III): V at one device point (3 float64) into out (device, 1
 * float64), one kernel launch, asynchronous on `stream`.  The whole GPU
 * shares the M cells; block partial sums are added by the last block to
 * finish, in fixed order (bitwise reproducible).
 *   mode 0: one workgroup of 256 threads per two compute units (the
 *           measured latency optimum: more workgroups cost more in launch
 *           and in the final sum than they save);
 *   mode 1: the paper's decomposition, 120 blocks x 256 threads, each thread
 *           taking every (120 x 256)-th cell (Sec. III, Eq. coalease).
 * Calls on one handle must not overlap (they share the block-partial
 * buffer): issue them on one stream.
 * Errors: ENV_E_ARG (NULL, bad mode), ENV_E_DEVICE. */
env_status env_cells_eval_single(env_cells* h, const double* point, double* out, int32_t mode,
                                 void* stream);

/* Resident single-point mode (the same moves without a launch or a copy call
 * per move): one kernel stays on the GPU with the workgroups of `mode` (as
 * in env_cells_eval_single) and takes positions from a mailbox in pinned
 * host memory; the host writes a position and waits for V, which the last
 * workgroup of the round writes back.  Same decomposition and fixed-order
 * sums as env_cells_eval_single, so the values are equal bit for bit.
 *   start: launch the kernel on a stream of the library's own (ENV_OK at
 *     once when it already runs with this mode and idle_s); the kernel
 *     exits by itself after idle_s seconds (0 < idle_s <= 3600) without a
 *     position, so one that is never stopped still ends;
 *   eval:  point and out are host pointers; returns when out is written
 *     (a kernel that left for lack of positions is launched again first);
 *     ENV_E_STATE before start, ENV_E_DEVICE when V does not arrive within
 *     timeout_s seconds (the kernel is then stopped);
 *   stop:  ask the kernel to exit and wait for it (env_cells_destroy does
 *     this too).
 * While the kernel runs it occupies its workgroups' compute units and
 * every other call on the device shares the rest; a device-wide wait
 * (hipDeviceSynchronize, torch.cuda.synchronize(), env_potential_export_image,
 * and HIP calls that wait for the whole device, such as hipFree) waits for
 * it to leave, so stop it first.  Calls on one handle must not overlap.
 * Errors: ENV_E_ARG (NULL, bad mode, idle_s or timeout_s), ENV_E_NOMEM,
 * ENV_E_DEVICE. */
env_status env_cells_resident_start(env_cells* h, int32_t mode, double idle_s);
env_status env_cells_resident_eval(env_cells* h, const double* point, double* out, double timeout_s);
env_status env_cells_resident_stop(env_cells* h);

void env_cells_destroy(env_cells* h);

void env_potential_destroy(env_potential* h);

const char* env_status_string(env_status s);

#ifdef __cplusplus
}
#endif

#endif /* ENV_POTENTIAL_H */
