/*
 * dyson.h -- C ABI of the MI355X library that computes the local Green's
 * function G_ii(i w_k) = [H(i w_k)^{-1}]_ii of the lattice Dyson matrix by the
 * Lanczos-based low-rank correction method (Carrier, Tang, Saad, Freericks,
 * arXiv:1102.3137).
 *
 * Problem statement (Sec. I, eq. (1)): on a hypercubic lattice with
 * nearest-neighbour bonds, H_ij = t for every bond and
 * H_ii = i w_k + mu - V_i - Sigma_i(i w_k).  Only diag(H^{-1}) is wanted.
 *
 * Conventions shared by every entry point
 *   - Sites are in natural order, x fastest: i = x + Lx*(y + Ly*z).
 *   - Complex arrays are interleaved (re, im) float64, frequency-major:
 *     element (k, i) of a [K][N] array sits at doubles 2*(k*N+i), 2*(k*N+i)+1.
 *   - Pointers named d_* are DEVICE pointers (hipMalloc'ed or any device
 *     memory visible to the plan's device); h_* are host pointers.
 *   - The caller owns every buffer passed in; the library never frees them
 *     and keeps none beyond the call, except the device buffers of a request
 *     submitted with DYSON_MEM_DEVICE (borrowed until it is finished or
 *     released).  The library owns contexts, plans and request handles.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     stream-ordered; a call returns after its work is enqueued and, for
 *     the solve entry points, after it has completed (they poll device-side
 *     convergence flags).
 *   - Errors are status codes; nothing throws across the ABI.  On error the
 *     output buffers are left untouched or partially written and must not
 *     be used; dyson_last_error() gives a message (thread-local).
 *   - Validation returns DYSON_EINVAL: dim not in {1,2,3}, any L < 1, K < 1
 *     or K > 65535 per call,
 *     w_k <= 0 (Im z_k <= 0), non-finite input, or Im(i w_k - Sigma_i) <= 0
 *     (Im(z_k - Sigma_i) <= 0); the last keeps Im H positive definite, so H
 *     and every principal submatrix are non-singular and the pivot-free
 *     factorizations below exist.
 */
#ifndef DYSON_MI355X_H
#define DYSON_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DYSON_OK = 0,
  DYSON_EINVAL = 1,      /* invalid argument or input value */
  DYSON_ENOMEM = 2,      /* device allocation failed */
  DYSON_EBREAKDOWN = 3,  /* Lanczos breakdown not cured by restarts */
  DYSON_ENOCONV = 4,     /* an inner solve hit its iteration cap */
  DYSON_EDEVICE = 5,     /* HIP runtime error */
  DYSON_EUNSUPPORTED = 6,/* valid request this build does not implement */
  DYSON_EBUSY = 7,       /* object still in use (a plan with live requests, a
                            context with live plans).  Admission never refuses a
                            request: one that does not fit the HBM budget waits
                            in the queue until memory frees up, or fails with
                            DYSON_ENOMEM if not even one frequency of it fits */
  DYSON_ECANCELLED = 8,  /* the request was cancelled */
  DYSON_ETIMEOUT = 9     /* dyson_wait returned before the request finished */
} dyson_status;

/* Lattice geometry and hopping (eq. (1)): chain, square (Z=4) or simple
 * cubic (Z=6) lattice.  periodic[a] = 1 wraps axis a (bond between sites
 * L_a - 1 and 0); such an axis needs L_a >= 3 and L_a a multiple of the leaf
 * edge, and its wrap plane (sites at coordinate L_a - 1) joins the interface
 * of the top correction level, which leaves every subdomain open. */
typedef struct {
  int dim;         /* 1, 2 or 3 */
  int L[3];        /* extents, unused axes = 1; x fastest */
  int periodic[3]; /* 0 open, 1 periodic; unused axes 0 */
  double t;        /* hopping: H_ij = t on each nearest-neighbour bond */
  double mu;       /* chemical potential in H_ii */
} dyson_lattice;

enum { DYSON_PART_NESTED = 0, DYSON_PART_SINGLE = 1 };
enum { DYSON_PREC_FP64 = 0, DYSON_PREC_MIXED = 1, DYSON_PREC_MIXED16 = 2 };

/* Method options.  Zero-initialise and set what you need; zero fields take
 * the defaults given in brackets. */
typedef struct {
  int leaf_edge;      /* subdomain edge s: separators at p with (p+1)%s==0 [16];
                         2..16 (chain, square), 2..6 (cubic: tiles of s^3 <= 216 sites).
                         0 takes the default: a plan is built before any input
                         exists, so the measured choice comes from dyson_autotune
                         on probe frequencies, whose result is then passed here */
  int partition;      /* DYSON_PART_NESTED: recursive bisection, alternating axes
                         (end of Sec. II.C); DYSON_PART_SINGLE: one level with
                         every separator at once (Fig. 1) [NESTED] */
  int precision;      /* DYSON_PREC_FP64; DYSON_PREC_MIXED: complex64 subdomain
                         factors in the inner preconditioner; DYSON_PREC_MIXED16:
                         complex32 (FP16 pairs) factors there; it needs
                         Im(z_k - Sigma_i) >= 2^-14 (the factor entries, bounded
                         by 1 / min Im H_ii, must fit FP16), else the solve
                         returns DYSON_EUNSUPPORTED.  Residuals, the
                         preconditioner arithmetic, Lanczos, re-orthogonalization
                         and the diagonal stay FP64 in every mode [FP64] */
  int max_rank;       /* cap on Lanczos steps per domain (truncated rank); 0 = full [0] */
  int extra_steps;    /* steps allowed beyond the interface size m (Sec. II.C):
                         the cap is m + max(extra_steps, ceil(m/8)) [10] */
  int max_inner_iters;/* iteration cap of each inner solve, 1..1000000 [2000] */
  double inner_tol;   /* relative residual of the inner solves [1e-14] */
  double lanczos_tol; /* stop when |r|_2 <= lanczos_tol*|u|_2 [1e-11] */
  uint64_t seed;      /* seed of the Lanczos start vectors [0x5eed] */
  int profile;        /* 1: time the dominant kernel (inner-solve update) with HIP
                         events on the call's stream; 2: every hot kernel class;
                         algorithmic bytes are counted for all classes [0] */
  int level_streams;  /* correction levels are independent (each adds its own
                         diag(X_l)); they run in up to this many concurrent
                         groups, each on its own HIP stream and workspace,
                         1 = one after the other, bottom-up.  Results do not
                         depend on timing; the group sums are added in a fixed
                         order [4].  HIP runs streams that share a hardware
                         queue one after another: with several solves or
                         server slots at once, give the process enough queues
                         (GPU_MAX_HW_QUEUES, read when the HIP runtime starts;
                         4 by default) */
  int check_sites;    /* sampled error estimate (report.est_rel_err): at this
                         many fixed sites (0..2; the first on the top-level
                         interface, the second inside a subdomain) the exact
                         G_ii = e_i^T H^{-1} e_i is also computed by solving
                         H x = e_i directly (eq. (14)) with the inner solver,
                         for every frequency; -1 = none [2] */
  int fault_step;     /* test hook for the breakdown path (Sec. II.A: the bilinear
                         "norm" r^T r can vanish): when > 0, every (domain,
                         frequency) item still open after fault_step Lanczos steps
                         is declared broken down at that step on its first
                         fault_attempts attempts, as if |r^T r| had vanished; the
                         item is then redone from a fresh start vector (report.
                         restarts), and DYSON_EBREAKDOWN results once the attempts
                         (3) are used up.  0 = off [0] */
  int fault_attempts; /* attempts on which fault_step trips, 0..3 [0] */
  double breakdown_tol; /* serious-breakdown threshold of the bilinear form: an
                         item whose new residual has |r^T r| <= breakdown_tol |r|_2^2
                         (so the next basis vector would have |q|_2^2 >=
                         1/breakdown_tol, amplifying rounding by as much) is
                         redone from a fresh start vector; each later attempt
                         uses a 100x smaller threshold [1e-4] */
  int interface_lanczos; /* 0: bilinear Lanczos on X (eqs. (8)-(12): two inner solves
                         per step, the diagonal streamed from the basis); 1: on the
                         Schur complement S = C - E^T B^{-1} E of each domain (from
                         eqs. (5)-(7)): one inner solve per step, exactly m steps, the
                         projected Hessenberg matrix H inverted once per (domain,
                         frequency) and diag(X) = diag(V H^{-1} V^T) with
                         V = [B^{-1} E P; P] [0] */
  int inner_graphs;     /* the inner solves' iterations between convergence polls
                         go to the GPU as captured HIP graphs of 8 iterations
                         (stencil, open-frequency compaction and update launches),
                         replayed for every later solve of the same shape; the
                         results are bit for bit those of direct launches.
                         0 = default (on), 1 = on, -1 = off (every kernel
                         launched directly).  Off while profiling and in
                         dyson_solve_noalloc [0] */
} dyson_opts;

/* Filled by dyson_solve when report != NULL. */
typedef struct {
  double t_total_ms;        /* host wall time of the call */
  int levels;               /* correction levels run */
  int max_rank_used;        /* largest Lanczos step count of any domain */
  long long lanczos_steps;  /* sum over (domain, frequency) of Lanczos steps */
  long long inner_iters;    /* sum over inner solves and items of iterations */
  int inner_iters_max;      /* worst single inner solve */
  int restarts;             /* breakdown restarts; in the interface form also the fresh
                               directions taken after an invariant subspace of S */
  int truncated;            /* 1 if any (domain, frequency) stopped at its step cap
                               (max_rank or m + extra) before the Krylov space of X
                               was exhausted: that result is not full rank */
  /* per-kernel timing (profile=1), HIP events on the call's stream around a
   * fixed pseudo-random one in sixteen of a class's launches, scaled to all
   * of them (kern_launches and kern_bytes count every launch):
   * 0 = inner-solve update + tile preconditioner (k_cocg_update),
   * 1 = inner-solve stencil (k_cocg_stencil), 2 = re-orthogonalization
   * update (k_cgs_update), 3 = re-orthogonalization products (k_cgs_dot) */
  double kern_ms[4];
  long long kern_launches[4];
  double kern_bytes[4];     /* algorithmic HBM bytes those launches moved */
  /* served requests (dyson_req_report): t_total_ms is arrival -> completion */
  double t_queue_ms;        /* arrival -> first frequency on the device */
  int batches;              /* device batches the request's frequencies ran in */
  size_t hbm_bytes;         /* largest workspace (device bytes) of those batches,
                               or of the call for dyson_solve */
  double est_rel_err;       /* largest relative difference, over the check sites
                               and frequencies, between G_ii and the direct solve
                               of H x = e_i (opts.check_sites); 0 when no check
                               ran (no correction level, or check_sites = -1) */
  int capped_items;         /* (domain, frequency) items stopped by their step cap
                               before exhaustion (truncated = capped_items > 0) */
} dyson_report;

typedef struct dyson_ctx dyson_ctx;
typedef struct dyson_plan dyson_plan;

/* Summary of a plan (the domain decomposition of eq. (4), recursively). */
typedef struct {
  int n_sites;        /* N */
  int n_tiles;        /* subdomain tiles (one leaf each) */
  int tile_sites;     /* padded sites per tile, s^dim */
  int levels;         /* correction levels (0 = the whole lattice) */
  int n_nodes[32];    /* correction domains per level */
  int max_m[32];      /* largest interface size m per level */
  long long sum_m[32];/* sum of m over the level's domains */
} dyson_plan_info;

/* Optional device allocator.  alloc returns device memory of `bytes` bytes
 * usable on `stream` (NULL on failure); free releases it.  Both may be called
 * from the library's worker threads. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, void* stream, void* user);
  void* user;
} dyson_allocator;

/* Context on one HIP device.  device = ordinal.  hbm_budget = device bytes
 * the serving slots may hold at once (0 = 90% of the device memory free at
 * creation); blocking calls allocate outside it.  allocator = NULL uses
 * hipMalloc/hipFree.  Teardown order: release requests, destroy plans, then
 * the context; dyson_destroy returns DYSON_EBUSY while plans made on it
 * exist (and a plan refuses destruction while it has requests), so no work
 * is in flight when the server stops. */
dyson_status dyson_create(dyson_ctx** ctx, int device, size_t hbm_budget,
                          const dyson_allocator* allocator);
dyson_status dyson_destroy(dyson_ctx* ctx);

/* Build the domain decomposition (host only, integer work; Fig. 1, eq. (4),
 * recursion at the end of Sec. II.C).  opts may be NULL for defaults. */
dyson_status dyson_plan_create(dyson_ctx* ctx, const dyson_lattice* lat,
                               const dyson_opts* opts, dyson_plan** plan);
/* DYSON_EBUSY while requests submitted on the plan are not yet released. */
dyson_status dyson_plan_destroy(dyson_plan* plan);
/* Gives back the device workspace that the plan's blocking calls (dyson_solve,
 * dyson_solve_z, dyson_solve_host, dyson_solve_schur and the stage entry
 * points) keep from one call to the next; the next such call allocates it
 * again.  The serving slots hold workspaces of their own, which the server
 * gives back when memory is short.  Must not overlap a blocking call on the
 * same plan from another thread. */
dyson_status dyson_plan_trim(dyson_plan* plan);
dyson_status dyson_plan_get_info(const dyson_plan* plan, dyson_plan_info* info);

/* Host copies of the plan's site maps, natural order, length N each:
 * h_depth[i]  = level at which site i becomes interface (separator), or, for
 *               subdomain-interior sites, the depth of their leaf;
 * h_is_sep[i] = 1 for separator sites, 0 for leaf-interior sites;
 * h_tile[i]   = the tile (leaf) holding site i (tiles numbered in the
 *               depth-first order of the domain tree). */
dyson_status dyson_plan_get_maps(const dyson_plan* plan, int* h_depth,
                                 int* h_is_sep, int* h_tile);

/* Interface size m and Lanczos step cap of every correction domain of a
 * level (domains in the order of dyson_correct_level's h_steps): the cap is
 * m + max(extra_steps, ceil(m/8)), or max_rank when that is smaller; a full-rank
 * domain takes between m and cap steps (eqs. (8)-(9): X has rank m).  In the
 * interface form (interface_lanczos = 1) the cap is m, and every domain takes
 * exactly m steps.  Either output may be NULL; each has
 * dyson_plan_info.n_nodes[level] entries. */
dyson_status dyson_plan_get_domains(const dyson_plan* plan, int level, int* h_m, int* h_cap);

/* Device memory a dyson_solve over K frequencies will allocate (bytes); the
 * serving slots hold the same per batch of K frequencies. */
dyson_status dyson_footprint(const dyson_plan* plan, int K, size_t* bytes);

/* Full hot path: diag(H(i w_k)^{-1}) for K frequencies.
 * d_V [N] f64; d_omega [K] f64 (w_k > 0); d_sigma [K][N] complex
 * (Sigma_i(i w_k)); d_G [K][N] complex output.  All device pointers.
 * Steps: assemble d_i (eq. (1)); factor the subdomain blocks and take
 * diag(B^{-1}) (eq. (13), first term); per level, bottom-up, bilinear Lanczos
 * on X = H^{-1} - blkdiag(B^{-1},0) (eqs. (7)-(12)) with the streaming
 * three-vector diagonal (after eq. (13)); combine and scatter. */
dyson_status dyson_solve(dyson_plan* plan, int K, const double* d_V,
                         const double* d_omega, const double* d_sigma,
                         double* d_G, void* stream, dyson_report* report);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): dyson_solve with no
 * allocation at all.  The workspace is carved from a fixed device array of
 * dyson_noalloc_max_bytes() bytes (256 MiB) that each device holds from the
 * first dyson_create on it until the process ends; inputs and output are the
 * caller's device buffers, as in dyson_solve.  The correction levels run one
 * after another on `stream` (the result equals dyson_solve with
 * level_streams = 1 bit for bit) and no profiling events are recorded.
 * Returns DYSON_EINVAL, before touching the device, when the plan's workspace
 * for K frequencies (dyson_noalloc_bytes) exceeds the array.  Every call on a
 * device uses the same array and leaves its contents behind: calls that
 * overlap on one device (threads, streams, plans) race and must be serialised
 * by the caller. */
dyson_status dyson_solve_noalloc(dyson_plan* plan, int K, const double* d_V,
                                 const double* d_omega, const double* d_sigma, double* d_G,
                                 void* stream, dyson_report* report);
/* Scratch bytes dyson_solve_noalloc needs for K frequencies of the plan. */
dyson_status dyson_noalloc_bytes(const dyson_plan* plan, int K, size_t* bytes);
/* Size of the per-device scratch array. */
size_t dyson_noalloc_max_bytes(void);

/* The host-to-host form of dyson_solve: h_V [N], h_omega [K], h_sigma [K][N]
 * and the output h_G [K][N] are HOST arrays (same layouts).  The inputs are
 * copied to a device staging block (allocated through the context's allocator
 * and freed before the call returns) on `stream`, the solve runs there, and G
 * is copied back before the call returns; report->t_total_ms includes the
 * copies.  Errors as dyson_solve, plus DYSON_ENOMEM if the staging block
 * (16 (2 K N + N) bytes) cannot be allocated; h_G is untouched on error. */
dyson_status dyson_solve_host(dyson_plan* plan, int K, const double* h_V, const double* h_omega,
                              const double* h_sigma, double* h_G, void* stream,
                              dyson_report* report);

/* The same hot path at complex energies z_k with Im z_k > 0 instead of the
 * Matsubara points i w_k: H_ii = z_k + mu - V_i - Sigma_i(z_k) (eq. (1)
 * continued off the imaginary axis, e.g. z_k = w_k + i eta on the real
 * axis).  d_z [K] complex; validation requires Im(z_k - Sigma_i) > 0.
 * z_k = i w_k gives exactly the dyson_solve result for w_k. */
dyson_status dyson_solve_z(dyson_plan* plan, int K, const double* d_V, const double* d_z,
                           const double* d_sigma, double* d_G, void* stream,
                           dyson_report* report);

/* Candidates of dyson_autotune (initialiser lists). */
#define DYSON_AUTOTUNE_EDGES_2D {8, 12, 16}
#define DYSON_AUTOTUNE_EDGES_3D {4, 5, 6}
#define DYSON_AUTOTUNE_LEVEL_STREAMS {1, 3, 4}
#define DYSON_AUTOTUNE_FORMS {0, 1}

/* The standard domain-decomposition inverse the paper compares against
 * (Sec. II.B, eqs. (4)-(6)): for a one-level decomposition (every separator in
 * one interface; DYSON_PART_SINGLE, or any plan with at most one correction
 * level) the Schur complement S = C - E^T B^{-1} E is formed explicitly (m x m
 * complex, m = interface sites) and inverted, and
 *   diag(H^{-1}) = diag(S^{-1}) on the interface,
 *   diag(B^{-1}) + diag(B^{-1} E S^{-1} E^T B^{-1}) inside the subdomains.
 * Arguments and layouts as dyson_solve (device pointers).  Every factor and
 * product is FP64 whatever opts.precision says.  Device memory: about
 * 16 K (m^2 + 64 m + T n_I S) bytes beyond the plan's workspace (T tiles of S
 * sites, n_I interface sites around one leaf), allocated and freed within the
 * call; DYSON_ENOMEM if that fails, DYSON_EUNSUPPORTED for a plan with more than
 * one correction level.  The report gives t_total_ms, hbm_bytes and
 * max_rank_used = m; with opts.profile set, kern_ms[0] is the event-timed
 * Gauss-Jordan inversion of S, kern_launches[0] its launches and kern_bytes[0]
 * its algorithmic flops (8 m^3 per frequency: m^3 complex multiply-adds). */
dyson_status dyson_solve_schur(dyson_plan* plan, int K, const double* d_V, const double* d_omega,
                               const double* d_sigma, double* d_G, void* stream,
                               dyson_report* report);

/* Measured choice of the tile shape and the form of the correction: for each
 * candidate leaf edge (DYSON_AUTOTUNE_EDGES_2D on chains and squares,
 * DYSON_AUTOTUNE_EDGES_3D on cubes; periodic axes keep only edges that divide
 * them), level-stream count (DYSON_AUTOTUNE_LEVEL_STREAMS) and form
 * (DYSON_AUTOTUNE_FORMS as interface_lanczos; only the X form when base sets
 * max_rank > 0), a plan solves the probe inputs (K frequencies, device
 * pointers as in dyson_solve) once after its workspace is allocated; the
 * fastest wins.  *best = base (NULL: defaults) with leaf_edge, level_streams
 * and interface_lanczos set; *rate = its site*freq/s.  The probe should be a
 * few representative frequencies of the intended workload. */
dyson_status dyson_autotune(dyson_ctx* ctx, const dyson_lattice* lat, const dyson_opts* base,
                            int K, const double* d_V, const double* d_omega,
                            const double* d_sigma, dyson_opts* best, double* rate);

/* ---- Stage entry points (the same kernels the solve runs), for testing ----
 * All pointers are device pointers; the plan's workspace for K frequencies
 * is (re)allocated as needed. */

/* eq. (1): d_d [K][N] complex = i w_k + mu - V_i - Sigma_i(i w_k). */
dyson_status dyson_assemble(dyson_plan* plan, int K, const double* d_V,
                            const double* d_omega, const double* d_sigma,
                            double* d_d, void* stream);

/* eq. (13), first term: for every leaf subdomain block B_s (the lattice
 * restricted to the leaf's sites), d_Gleaf[k][i] = [B_s(w_k)^{-1}]_ii for
 * leaf sites and 0 for separator sites.  d_d as produced by dyson_assemble. */
dyson_status dyson_leaf_diag(dyson_plan* plan, int K, const double* d_d,
                             double* d_Gleaf, void* stream);

/* eqs. (10)-(12): d_u = X_l d_q for every correction domain of level l at
 * once, X_l = H_l^{-1} - blkdiag(B_l^{-1}, 0) with H_l the lattice restricted
 * to each level-l domain and B_l its subdomains.  d_q [K][N] complex; entries
 * outside level-l domains are ignored, those of d_u are set to 0. */
dyson_status dyson_xmatvec(dyson_plan* plan, int level, int K,
                           const double* d_d, const double* d_q, double* d_u,
                           void* stream);

/* One level of the correction: bilinear Lanczos on X_l for every level-l
 * domain and frequency, adding diag(Q T Q^T) into d_Gacc [K][N] (complex,
 * accumulated in place).  h_steps [K*n_nodes] (may be NULL) receives the
 * Lanczos steps per (frequency, domain), domain-fastest. */
dyson_status dyson_correct_level(dyson_plan* plan, int level, int K,
                                 const double* d_d, double* d_Gacc,
                                 int* h_steps, void* stream);

/* ---- Serving: asynchronous requests with continuous batching ----
 * A request is one dyson_solve's worth of work (eq. (1) inputs for K
 * frequencies of one plan).  Requests are cut into runs of frequencies
 * (frequencies are independent problems); a pool of slots, each with its own
 * HIP stream and workspace, takes the oldest waiting frequencies together
 * with those of every other waiting request on the same plan, up to
 * max_batch_freqs and as far as the HBM budget allows, and runs them as one
 * batch.  Requests that arrive while batches run join the next batch a slot
 * forms; slots run concurrently on the device.  Results do not depend on how
 * requests were batched: every (domain, frequency) item is computed the
 * same way alone or in a mix (its start vector is keyed by the bits of w_k).
 *
 * mem = DYSON_MEM_DEVICE: V, omega, sigma and G are device pointers that the
 * library borrows until the request is finished or released; inputs must be
 * complete (stream-synchronized) when dyson_submit is called.
 * mem = DYSON_MEM_HOST: V, omega, sigma are host arrays copied before
 * dyson_submit returns; G is a host array written when the request finishes.
 * Inputs are validated in dyson_submit (DYSON_EINVAL, as for dyson_solve).
 * The first dyson_submit on a context starts its server. */
enum { DYSON_MEM_DEVICE = 0, DYSON_MEM_HOST = 1 };
typedef struct dyson_req dyson_req;

/* Slots (1..8, default 3) and frequencies per batch (1..4096, default 256);
 * call before the first dyson_submit on the context. */
dyson_status dyson_serve_config(dyson_ctx* ctx, int slots, int max_batch_freqs);
dyson_status dyson_submit(dyson_plan* plan, int K, const double* V, const double* omega,
                          const double* sigma, double* G, int mem, dyson_req** req);
/* A request at complex energies z [K] complex (as dyson_solve_z); requests of
 * both kinds on one plan share batches. */
dyson_status dyson_submit_z(dyson_plan* plan, int K, const double* V, const double* z,
                            const double* sigma, double* G, int mem, dyson_req** req);
/* *done = 1 once the request has finished (successfully or not). */
dyson_status dyson_poll(dyson_req* req, int* done);
/* Block until the request finishes or timeout_s (< 0: no limit) passes.
 * Returns the request's final status, or DYSON_ETIMEOUT. */
dyson_status dyson_wait(dyson_req* req, double timeout_s);
/* Drop the request's frequencies that are still queued; those already on
 * the device finish.  The request ends with DYSON_ECANCELLED and G is
 * unspecified.  No effect on a finished request. */
dyson_status dyson_cancel(dyson_req* req);
/* Timing and statistics of a finished request (DYSON_EBUSY before). */
dyson_status dyson_req_report(dyson_req* req, dyson_report* report);
/* Cancel if unfinished, wait until none of its frequencies is on the device,
 * and free the handle. */
dyson_status dyson_release(dyson_req* req);

/* Several plans in one blocking call (e.g. lattices of different sizes and
 * dimensions, each with its own frequencies): request i = plan i with Ks[i]
 * frequencies and DEVICE arrays d_V[i] [N_i], d_omega[i] [K_i], d_sigma[i]
 * [K_i][N_i] and d_G[i] [K_i][N_i] (layouts as dyson_solve).  The inputs may
 * be written on `stream`: it is synchronized first.  The requests go through
 * the context's server as one arrival, so they are split into frequency
 * batches by the HBM budget and run concurrently in its slots (continuous
 * batching); each G equals its own dyson_submit result bit for bit.  All plans
 * belong to one context.  Returns when every request has finished: the first
 * error of any of them, with every request released; reports[i] (may be NULL)
 * as dyson_req_report. */
dyson_status dyson_solve_batch(int n, dyson_plan* const* plans, const int* Ks,
                               const double* const* d_V, const double* const* d_omega,
                               const double* const* d_sigma, double* const* d_G, void* stream,
                               dyson_report* reports);

const char* dyson_last_error(void);
const char* dyson_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DYSON_MI355X_H */
