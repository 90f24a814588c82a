/*
 * spaqr.h -- C ABI of the MI355X spaQR engine.
 *
 * spaQR (sparsified QR) computes an approximate factorization Q^T A W^{-1} ~ I
 * of a sparse square matrix A, where Q is a product of orthogonal factors and
 * W a product of orthogonal and upper-triangular factors, by eliminating a
 * nested-dissection tree level by level and compressing separator interfaces
 * to a tolerance eps (Algorithm 2, Sections 2.4-2.8).  M^{-1} = W^{-1} Q^T is
 * then used as a preconditioner inside GMRES (Section 4).
 *
 * Conventions for every call:
 *   - every call returns a spaqr_status; no exception crosses the ABI;
 *   - on error the output arguments are left untouched;
 *   - matrices are FP64 CSR on the host, 0-based, columns sorted, no
 *     duplicates;
 *   - dense vectors are column-major n x nrhs with leading dimension ld >= n;
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *     device memory (for example a PyTorch CUDA/HIP tensor's data pointer);
 *   - one thread uses a handle at a time; distinct handles are independent.
 */
#ifndef SPAQR_H
#define SPAQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
typedef int spaqr_status;
#define SPAQR_OK 0          /* success */
#define SPAQR_ENOCONV 1     /* warning: GMRES hit maxit; x holds the best iterate */
#define SPAQR_EINVAL (-1)   /* invalid argument (malformed CSR, bad ordering, ...) */
#define SPAQR_ENOMEM (-2)   /* a host or device allocation failed */
#define SPAQR_ESINGULAR (-3)/* a front produced an exactly zero diagonal in R_ss */
#define SPAQR_EDEVICE (-4)  /* a HIP runtime call failed, or no GPU is present */

/* Static, NUL-terminated description of a status code. */
const char* spaqr_status_string(int status);
/* Message of the last failed call on the calling thread ("" if none).  The
 * string stays valid until the next call on that thread. */
const char* spaqr_last_error(void);

/* ------------------------------------------------------------------ matrix */
/* Host FP64 CSR (caller-owned; read only during the call that receives it). */
typedef struct {
  int64_t n;               /* rows = columns */
  int64_t nnz;             /* stored entries */
  const int64_t* rowptr;   /* n + 1 entries */
  const int32_t* col;      /* nnz entries, sorted within each row */
  const double* val;       /* nnz entries */
} spaqr_csr;

/* ---------------------------------------------------------------- ordering */
/* Geometric modified nested dissection of a dim-dimensional box grid with
 * sides[0..dim-1] points and lexicographic point index x + n0*y (+ n0*n1*z)
 * (Section 2.3; geometric partitioning of A^T A for grids, Section 4).
 * Separators are two grid layers thick (they must cut the graph of A^T A);
 * a box splits on its longest axis (ties to the lowest axis) at
 * m = lo + floor((w-2)/2), separator {m, m+1}; separator interfaces are the
 * classes of the pair of level-k ancestors of the deepest nodes touched on
 * each side (modified ND, Figs. mnd and mnd_multilvl).
 * nlevels <= 0 selects ceil(log2(N/64)) (Section 4, setup), capped at the
 * deepest tree the grid allows (every box above the leaves needs a longest
 * extent >= 4); an explicit nlevels deeper than that is EINVAL.
 * Errors: EINVAL if dim is not 2 or 3, a side is < 1, or a box above the
 * leaves has its longest extent < 4.  *out is library-owned; release it with
 * spaqr_ordering_free. */
typedef struct spaqr_ordering spaqr_ordering;
spaqr_status spaqr_order_grid(int dim, const int32_t sides[3], int nlevels,
                              spaqr_ordering** out);
/* Algebraic modified nested dissection of a square sparse matrix without a
 * grid (Section 2.3, Fig. mnd; the paper partitions such matrices with a
 * hypergraph partitioner, here the graph of A^T A is bisected instead).
 * Graph: i ~ j (i != j) iff some row of A holds entries in columns i and j.
 * A node's vertex set splits between two far vertices of its induced
 * subgraph: r starts at the smallest vertex and moves up to four times to
 * the smallest vertex of its last BFS level while that lengthens the level
 * structure; u is then the smallest vertex of r's last level.  Each vertex
 * of r's component gets the key d_r - d_u (BFS distances); the separator is
 * the key pair {t, t+1} minimizing (|#low - #high|, its size, t), low =
 * keys below t, high = keys above t+1 plus the other components.  The pair
 * is then thinned: its vertices with no high neighbour join the low part,
 * then those with no low neighbour join the high part.  A separator
 * vertex's stage-k interface is the pair of
 * level-k ancestors of the deepest common ancestors of its neighbours' nodes
 * on each side.  Only A's pattern is read (A->val may be NULL); rows are
 * clustered like columns.  nlevels <= 0 selects ceil(log2(N/64)), capped at
 * the deepest tree whose nodes above the leaves all split (key range >= 3);
 * an explicit deeper nlevels is EINVAL.  Errors: EINVAL for a NULL or
 * inconsistent CSR or a column index outside [0, n).  *out is
 * library-owned (spaqr_ordering_free); the result is used like that of
 * spaqr_order_grid. */
spaqr_status spaqr_order_graph(const spaqr_csr* A, int nlevels, spaqr_ordering** out);
void spaqr_ordering_free(spaqr_ordering* ord);
int64_t spaqr_ordering_n(const spaqr_ordering* ord);
int spaqr_ordering_levels(const spaqr_ordering* ord);
/* perm[new] = old, n entries (host buffer, caller-allocated). */
spaqr_status spaqr_ordering_perm(const spaqr_ordering* ord, int64_t* perm);
/* Clusters of stage k (1 <= k <= L): the nodes of level > k are eliminated;
 * a node of level k is one cluster; separators of level < k are split into
 * interfaces.  Each cluster is a contiguous range [start, end) of perm.
 * Query the count with spaqr_ordering_num_clusters, then fill caller arrays
 * of that length (any of them may be NULL). */
int64_t spaqr_ordering_num_clusters(const spaqr_ordering* ord, int stage);
spaqr_status spaqr_ordering_clusters(const spaqr_ordering* ord, int stage,
                                     int64_t* start, int64_t* end,
                                     int64_t* node, int32_t* level);
/* parent[c] = index of the stage-(k-1) cluster that contains stage-k cluster
 * c, or -1 if c is eliminated at stage k (Section 2.7 merge). stage >= 2. */
spaqr_status spaqr_ordering_merge_parents(const spaqr_ordering* ord, int stage,
                                          int64_t* parent);

/* ----------------------------------------------------------------- options */
typedef struct {
  double eps;      /* sparsification tolerance (ratio rule |R_ii|/|R_11|), >= 0 */
  int skip;        /* levels above the leaves without sparsification (default 2) */
  int scale;       /* 1: block-diagonal scaling of the interfaces before their
                      sparsification (Section 2.6, the default); 0: the
                      sparsification without scaling of Section 2.5, with
                      sigma = 1/sigma_min(A_p) of Lemma 1 and a Householder QR
                      of the fine unknowns (interfaces of at most 1024
                      unknowns and 512 neighbour blocks, else SPAQR_EINVAL) */
  int precision;   /* 32: FP32 blocks and factors, 64: FP64 (default 32) */
  int restart;     /* GMRES restart length (default 100) */
  int maxit;       /* GMRES maximum Arnoldi steps (default 1000) */
} spaqr_opts;
spaqr_opts spaqr_opts_default(void);

/* ---------------------------------------------------------------- symbolic */
/* Host-only symbolic analysis of A's pattern under an ordering: per stage the
 * cluster block pattern, the fronts with their row and column sets and
 * colours, the fill, and the interface colouring (no device work).
 * Errors: EINVAL on a malformed CSR, a size mismatch, or a zero diagonal
 * block pattern.  Release with spaqr_symbolic_free. */
typedef struct spaqr_symbolic spaqr_symbolic;
spaqr_status spaqr_analyze(const spaqr_csr* A, const spaqr_ordering* ord,
                           const spaqr_opts* opts, spaqr_symbolic** out);
void spaqr_symbolic_free(spaqr_symbolic* sym);

/* Serialized per-stage symbolic information (for tests and tools).
 * what = 0: block pattern at stage start, pairs (row, col) sorted;
 *        1: block pattern after the fronts (with fill), pairs sorted;
 *        2: fronts in cluster order, each record
 *           [cluster, colour, |n1|, n1..., |cols|, cols...] (cols excludes
 *           the front itself);
 *        3: interface colours, pairs (cluster, colour) in cluster order
 *           (empty if the stage does not sparsify).
 * Call with buf = NULL to get the length in *len; then with cap >= *len. */
spaqr_status spaqr_symbolic_stage_info(const spaqr_symbolic* sym, int stage, int what,
                                       int32_t* buf, int64_t cap, int64_t* len);

/* ------------------------------------------------------------------ factor */
/* Numeric factorization on the HIP stream `hip_stream` (a hipStream_t; NULL
 * means the default stream).  The handle owns all device factors and a
 * device copy of A for the SpMV of spaqr_solve.  The ordering must have been
 * built for A's grid (same n).
 * Errors: EINVAL (bad arguments, ord n != A n, opts invalid), ENOMEM,
 * ESINGULAR (an exactly zero diagonal in some R_ss), EDEVICE. */
typedef struct spaqr_handle spaqr_handle;
spaqr_status spaqr_factor(const spaqr_csr* A, const spaqr_ordering* ord,
                          const spaqr_opts* opts, void* hip_stream,
                          spaqr_handle** out);
/* Same, reusing a symbolic analysis made for the same pattern and ordering. */
spaqr_status spaqr_factor_symbolic(const spaqr_csr* A, const spaqr_symbolic* sym,
                                   const spaqr_opts* opts, void* hip_stream,
                                   spaqr_handle** out);

/* Device-resident copies of a CSR matrix (HIP device pointers), laid out
 * exactly like the host spaqr_csr passed beside them. */
typedef struct {
  const int64_t* rowptr;
  const int32_t* col;
  const double* val;
} spaqr_csr_dev;

/* Factorization whose matrix values are already resident on the device.
 * A_pattern supplies n, nnz, rowptr and col on the host (its val may be NULL);
 * A_dev holds the same CSR in device memory; sym is an analysis of that
 * pattern.  The values never cross PCIe: the column scaling and the scatter
 * into the stage blocks run on the device, and the CSR is copied device to
 * device for the SpMV (A_dev may be freed after the call).
 * Errors: as spaqr_factor; EINVAL also for a numerically zero column. */
spaqr_status spaqr_factor_device(const spaqr_csr* A_pattern, const spaqr_csr_dev* A_dev,
                                 const spaqr_symbolic* sym, const spaqr_opts* opts,
                                 void* hip_stream, spaqr_handle** out);

/* Several factorizations advanced together, stage by stage (cross-request
 * batching; the paper factors one matrix at a time): at every stage the
 * fronts, scalings and sparsifications of all nprob problems share one
 * launch per phase.  Problem i: A[i] (host CSR; its values are read only if
 * Ad is NULL or Ad[i] is NULL), Ad[i] (device copy as in
 * spaqr_factor_device, or NULL), sym[i] (an analysis of A[i]'s pattern that
 * must outlive the handle).  opts (NULL: defaults) applies to all; all run on
 * hip_stream.  out[i] receives problem i's handle.  Returns OK when every
 * problem factored; otherwise the status of the first that failed, with
 * out[i] = NULL exactly for the failed ones (the others are valid handles
 * the caller frees).  EINVAL for bad arguments before any work. */
spaqr_status spaqr_factor_batch(int nprob, const spaqr_csr* const* A, const spaqr_csr_dev* const* Ad,
                                const spaqr_symbolic* const* sym, const spaqr_opts* opts,
                                void* hip_stream, spaqr_handle** out);

/* x = M^{-1} b = D_c P^T W^{-1} Q^T P b for nrhs columns (Section 2.8).
 * b and x: n x nrhs column-major with leading dimension ld; device pointers
 * if on_device != 0, else host pointers.  b and x may alias.  Runs on the
 * handle's stream and returns after the result is complete.
 * Errors: EINVAL (NULL pointers, nrhs < 1, ld < n), EDEVICE. */
spaqr_status spaqr_apply(spaqr_handle* h, const double* b, double* x,
                         int64_t nrhs, int64_t ld, int on_device);

/* The apply of spaqr_apply for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  b and x are device pointers (n x nrhs, column-major, leading
 * dimension ld >= n; they may alias).  The only workspace, the permuted
 * vectors, is a fixed array of 2^23 doubles (64 MiB) that the library holds on
 * every GPU it runs on until the process ends (spaqr_apply_noalloc_max()
 * returns that size): n * nrhs must not exceed it.  The call allocates
 * nothing, enqueues the apply on the handle's stream and returns without
 * waiting; the result is complete once that stream has passed it.  Every
 * call on one GPU uses that GPU's one array, so calls whose work overlaps on
 * one GPU (on different streams, or from several threads) race; calls on one
 * stream are ordered.  The array's contents are overwritten by every call.
 * Errors: EINVAL (NULL pointer, nrhs < 1, ld < n, n * nrhs above the array,
 * a handle without a complete factorization), EDEVICE. */
spaqr_status spaqr_apply_noalloc(spaqr_handle* h, const double* b, double* x,
                                 int64_t nrhs, int64_t ld);
int64_t spaqr_apply_noalloc_max(void);

/* Per-column outcome of spaqr_solve. */
typedef struct {
  int32_t iterations;  /* Arnoldi steps taken */
  int32_t converged;   /* 1 if ||A x - b|| / ||b|| <= tol */
  double relres;       /* true relative residual of the returned x */
  double seconds;      /* wall time of the whole solve call */
} spaqr_solve_info;

/* Right-preconditioned flexible GMRES in FP64 on the device, x0 = 0, until
 * ||A x - b|| / ||b|| <= tol for each column (Section 4).  Layout as in
 * spaqr_apply; info (host, nrhs entries, may be NULL) receives per-column
 * results.  Returns ENOCONV if some column hit maxit (x then holds its best
 * iterate), EINVAL, EDEVICE. */
spaqr_status spaqr_solve(spaqr_handle* h, const double* b, double* x,
                         int64_t nrhs, int64_t ld, int on_device, double tol,
                         spaqr_solve_info* info);

/* FGMRES for several handles at once (all made on one stream): the Arnoldi
 * steps of every column of every problem advance together and each step's
 * preconditioner applies and SpMVs run one launch per phase for all problems
 * (Section 4's method per column, batched across requests).  Problem i:
 * b[i] and x[i] hold nrhs[i] columns with leading dimension n_i (device
 * pointers if on_device != 0, else host), solved to tol[i].  info (may be
 * NULL) receives sum(nrhs) entries, problem by problem.  Returns ENOCONV if
 * some column hit maxit (the largest restart and maxit of the handles
 * apply), EINVAL (bad arguments, handles on different streams), EDEVICE. */
spaqr_status spaqr_solve_batch(int nprob, spaqr_handle* const* h, const double* const* b,
                               double* const* x, const int64_t* nrhs, int on_device,
                               const double* tol, spaqr_solve_info* info);

/* Factorization statistics. */
typedef struct {
  int64_t n;                 /* unknowns */
  int32_t levels;            /* nested-dissection levels L */
  int32_t precision;         /* 32 or 64 */
  int64_t factor_bytes;      /* bytes of stored factors (V, tau, T, R, U, Q) */
  int64_t top_separator;     /* unknowns of the root separator after every sparsification
                                that had neighbours to compress against (its size at the
                                start of stage 2; the root front's size if L = 1) */
  int64_t fronts;            /* number of fronts factored */
  int64_t interfaces_sparsified;
  double flops_front;        /* algorithmic flops: front QR + trailing update */
  double flops_scale;        /* scaling QR + block products */
  double flops_sparsify;     /* CPQR */
  double ms_symbolic;        /* host symbolic analysis */
  double ms_factor;          /* numeric factorization wall time */
  double ms_phase[4];        /* front, scale, sparsify, merge (device time) */
} spaqr_stats_t;
spaqr_status spaqr_stats(const spaqr_handle* h, spaqr_stats_t* out);

/* Statistics of one stage k of a completed factorization (the quantities of
 * the paper's Section 4.3 experiments, per stage).  Device times come from
 * HIP events around the stage's phases; in a batched factorization the
 * phases of one stage are shared by the problems advanced together, so the
 * times are those of the whole batch's launches.
 * Errors: EINVAL (NULL argument, stage outside 1..L, factorization not
 * complete). */
typedef struct {
  int32_t stage;              /* k */
  int32_t sparsified;         /* 1 if the stage scaled and sparsified its interfaces */
  int32_t fronts;             /* fronts (separators or leaves of level k) factored */
  int32_t max_front_rows;     /* largest m_s = |s| + sum of its row neighbours */
  int32_t max_front_pivots;   /* largest n_s = |s| */
  int32_t interfaces;         /* interfaces scaled and sparsified (|p| > 0) */
  int32_t max_nbr_cols;       /* largest m_p, the columns of C_p = [A_np^T | A_pn] */
  int32_t iface_size_q1;      /* quartiles and maximum of |p| before sparsification */
  int32_t iface_size_median;
  int32_t iface_size_q3;
  int32_t iface_size_max;
  int32_t pad;
  int64_t front_pivots;       /* sum of n_s */
  int64_t iface_unknowns_in;  /* sum of |p| before the sparsification */
  int64_t iface_unknowns_out; /* sum of the ranks r_p */
  int64_t nbr_cols;           /* sum of m_p */
  int64_t top_separator;      /* unknowns of the root separator at the start of the stage */
  int64_t factor_bytes;       /* bytes of factors the stage stored */
  double flops_front;         /* algorithmic flops of the phases (as in spaqr_stats_t) */
  double flops_scale;
  double flops_sparsify;
  double ms_front;            /* device time of the phases */
  double ms_scale;
  double ms_sparsify;         /* CPQRs and the dense interface operators */
  double ms_merge;
} spaqr_stage_stats_t;
spaqr_status spaqr_stage_stats(const spaqr_handle* h, int stage, spaqr_stage_stats_t* out);

/* The interfaces sparsified at stage k, four int32 per interface:
 * (cluster, |p|, m_p, r_p) in cluster order (Section 2.5-2.6 sizes and the
 * rank the ratio rule chose).  Same query protocol as
 * spaqr_symbolic_stage_info (len counts int32 entries). */
spaqr_status spaqr_stage_interfaces(const spaqr_handle* h, int stage, int32_t* buf, int64_t cap,
                                    int64_t* len);

/* Residual history of the handle's last spaqr_solve, first column: the
 * FGMRES estimate |g_{j+1}| / ||b|| after every Arnoldi step j, then the
 * true relative residual of the returned x as the last entry.  Same query
 * protocol (len counts doubles).  Errors: EINVAL. */
spaqr_status spaqr_solve_history(const spaqr_handle* h, double* buf, int64_t cap, int64_t* len);

/* Sizes of the stage-k clusters after stage k's sparsification (ranks of
 * sparsified interfaces; unchanged sizes otherwise).  Same query protocol as
 * spaqr_symbolic_stage_info. */
spaqr_status spaqr_stage_sizes(const spaqr_handle* h, int stage, int32_t* buf,
                               int64_t cap, int64_t* len);

/* Per-kernel timing (HIP events recorded on the launching stream around every
 * launch) and the algorithmic flops/bytes of those launches.  enable(1, only)
 * clears the table and starts recording every kernel (only == NULL), just
 * the kernel named `only`, or, when `only` ends in '*', every name with that
 * prefix; enable(0, NULL) stops.  Kernel names:
 * "front_qr", "scale_qr", "scale_blocks", "sparsify", "sparsify_unscaled"
 * (the sparsification without scaling, scale = 0), "copy",
 * "apply_front_fwd", "apply_front_bwd", "apply_iface_fwd", "apply_iface_bwd".
 * Block copies are recorded under "copy" and under their role
 * ("copy_front_gather", "copy_front_scatter", "copy_front_pack",
 * "copy_scale_gather", "copy_scale_pack", "copy_merge"), the role records
 * counting tiles in place of flops.
 * Host phases of the batched driver are recorded the same way (wall time as
 * the duration, zero work) under names starting with "host_", e.g.
 * "host_setup", "host_wait_gpu", "host_solve_setup", "host_solve_krylov".
 * Unknown names report zero launches. */
spaqr_status spaqr_profile_enable(int on, const char* only);
spaqr_status spaqr_profile_query(const char* kernel, int64_t* launches, double* total_ms,
                                 double* flops, double* bytes);

/* Launches of one kernel family since the process started (or since the
 * last reset), counted by the launchers whatever the profiler's state: the
 * kernel template's name, e.g. "k_qr_reg", "k_qr", "k_trail", "k_scale_small",
 * "k_scale_right", "k_cpqr_reg", "k_cpqr_coop", "k_sparsify",
 * "k_ap_front_fwd_wy", "k_ap_front_bwd_reg", "k_ap_iface_fwd",
 * "k_ap_iface_bwd", "k_ap_iface_dense", "k_ap_iface_dense_big",
 * "k_sparsify_unscaled", "k_iface_form", "k_copy".  Tests use
 * it to show which kernel paths a case exercised.  kernel == NULL resets
 * every count (and writes 0).  Unknown names give 0.  Errors: EINVAL if
 * count is NULL. */
spaqr_status spaqr_kernel_launches(const char* kernel, int64_t* count);

/* Releases all host and device memory of the handle.  NULL is a no-op. */
void spaqr_free(spaqr_handle* h);

/* Kernel dispatch thresholds (tile and block-size schedule), process-wide.
 * They choose which kernel runs each block, never what is computed: every
 * setting gives the same factorization up to rounding order.
 *   qr_reg_max_rows   fronts and scaling blocks of at most this many rows
 *                     are factored by the register-panel QR, taller ones by
 *                     the LDS-panel QR (256, 512 or 1024; default 1024);
 *   split_rows,       a front with more rows than split_rows, or at least
 *   split_cols        split_cols trailing columns, is factored as its pivot
 *                     block alone, its trailing columns updated slice by
 *                     slice (default 1024 and 1024);
 *   cpqr_reg          1: interfaces whose columns fit in registers take the
 *                     register CPQR; 0: they take the other kernels
 *                     (default 1);
 *   cpqr_coop         1: interfaces beyond the register CPQR take the
 *                     cooperative multi-workgroup CPQR when its workgroups
 *                     can be co-resident; 0: they take the single-workgroup
 *                     LDS kernel (up to 64 FP32 / 32 FP64 unknowns) or the
 *                     generic one (default 1);
 *   scale_small       scaling blocks of at most this size in both
 *                     dimensions take the fused LDS kernel (0, 16, 32 or 64;
 *                     default 64);
 *   iface_dense       interfaces of at most this many unknowns get dense
 *                     apply operators (0, 16, 32 or 64; default 64);
 *   trail_mfma        1: the trailing columns of a split front are updated
 *                     on the matrix cores, 64 reflectors and 64 columns at a
 *                     time; 0: by the vector-ALU slice kernel (default 1);
 *   cpqr_dd           1: FP32 interfaces of at most 64 unknowns whose
 *                     columns fit one workgroup take the CPQR with
 *                     downdated column norms (exact recomputation when a
 *                     norm has lost three digits, exact norms for the rank
 *                     rule), every interface of a colour in one launch;
 *                     2: as 1, with the interfaces of consecutive colours
 *                     in one launch, each waiting only for its adjacent
 *                     interfaces of earlier colours (the same results);
 *                     0: they take the exact-norm kernels above (default 2);
 *   cpqr_team         1: FP32 interfaces of 65-896 unknowns beyond one
 *                     workgroup take the team CPQR (a team of co-resident
 *                     workgroups per interface, all columns in registers,
 *                     downdated norms as for cpqr_dd); 2: so do those of at
 *                     most 64 unknowns with at least 16384 columns; 0: they
 *                     take the cooperative kernel (default 2).
 * spaqr_set_tuning(NULL) restores the defaults.  Set it only while no
 * factorization or apply is in flight.  Errors: EINVAL for a value outside
 * the ranges above. */
typedef struct {
  int qr_reg_max_rows;
  int split_rows, split_cols;
  int cpqr_reg;
  int cpqr_coop;
  int scale_small;
  int iface_dense;
  int trail_mfma;
  int cpqr_dd;
  int cpqr_team;
} spaqr_tuning;
spaqr_status spaqr_set_tuning(const spaqr_tuning* t);
spaqr_status spaqr_get_tuning(spaqr_tuning* t);

/* Returns to the HIP runtime the memory the library keeps for reuse across
 * calls (its cache of freed device blocks, its pool of pinned staging
 * buffers) and the profiler's pending events, after a device
 * synchronization.  Memory still owned by live handles, servers, analyses or
 * orderings is untouched.  Meant for process teardown: call it after freeing
 * every object and before the HIP runtime unloads (the Python binding calls
 * it from an interpreter exit hook), so that no HIP call of this library runs
 * during static destruction.  The library stays usable afterwards; the
 * caches refill on demand.  Never fails. */
void spaqr_finalize(void);

/* ----------------------------------------------------------------- serving */
/* Continuous-batching request loop (no counterpart in the paper, which
 * factors one matrix at a time).
 *
 * spaqr_server_create: mem_budget = bytes of device memory the resident
 *   requests may use (by the estimate below); hip_stream = the stream every
 *   request's work runs on (NULL: the default stream).  The server owns the
 *   factors of its requests.
 * spaqr_submit: copies A, the ordering, the options (NULL: defaults) and
 *   b (host, n x nrhs column-major, ld = n), runs the symbolic analysis
 *   (host) and queues the request; *ticket names it.  The request's
 *   estimated memory is spaqr_estimate_bytes of that analysis.  Returns
 *   ENOMEM if that estimate alone exceeds the budget, EINVAL on bad
 *   arguments or a malformed matrix.
 * spaqr_server_step: one round of the loop: (1) admits queued requests in
 *   arrival order while the sum of the resident requests' estimates stays
 *   within the budget (matrix upload and set-up);
 *   (2) advances every admitted request that is still factoring by one stage,
 *   all of them together: their fronts, scalings and sparsifications share
 *   one launch per phase whatever stage each one is at, so a request that
 *   arrives while others are half-way joins their batch; (3) solves every
 *   request whose factorization is complete, all its right-hand sides at once
 *   (multi-RHS FGMRES to its tol), in groups of similar size that share one
 *   batched FGMRES (at most 64 right-hand sides and 2^23 padded vector
 *   entries per group), and retires it.  *active (may be NULL)
 *   receives the number of requests still queued or in flight.  A request
 *   whose factorization fails (zero column, zero R_ss diagonal) is retired
 *   with that status; the others continue.
 * spaqr_poll: SPAQR_PENDING (2) while the ticket is not done; afterwards the
 *   request's final status (OK, ENOCONV, or the error it failed with), with
 *   x (host, n x nrhs, ld = n) and info (nrhs entries) filled when solved.
 *   A ticket can be polled to completion once.
 * One thread drives a server at a time. */
#define SPAQR_PENDING 2
typedef struct spaqr_server spaqr_server;
spaqr_status spaqr_server_create(size_t mem_budget, void* hip_stream, spaqr_server** out);
spaqr_status spaqr_submit(spaqr_server* srv, const spaqr_csr* A, const spaqr_ordering* ord,
                          const spaqr_opts* opts, const double* b, int64_t nrhs,
                          double tol, uint64_t* ticket);
spaqr_status spaqr_server_step(spaqr_server* srv, int* active);
spaqr_status spaqr_poll(spaqr_server* srv, uint64_t ticket, double* x,
                        spaqr_solve_info* info);
void spaqr_server_destroy(spaqr_server* srv);
/* Occupancy of a server: requests queued (submitted, not admitted),
 * requests resident (admitted, factoring or waiting for their solve), and
 * the sum of the resident requests' estimates in bytes (any pointer may be
 * NULL).  Errors: EINVAL for a NULL server. */
spaqr_status spaqr_server_status(const spaqr_server* srv, int64_t* queued, int64_t* resident,
                                 size_t* bytes);

/* Upper bound on the device memory, in bytes, that a factorization of the
 * analysed matrix (with opts->precision, NULL: defaults) and a solve of nrhs
 * right-hand sides hold at their peak.  Every block, front and interface is
 * sized as if nothing were compressed (ranks never exceed cluster sizes):
 * the persistent factors and apply lists, the largest stage workspace, two
 * stage block pools, the descriptor lists, each bounded by the arena
 * reservations the library makes for them, plus the FGMRES bases of nrhs
 * columns (2 * restart + 8 vectors each).  The server admits requests by it.
 * Errors: EINVAL (NULL argument, nrhs < 1, precision not 32 or 64). */
spaqr_status spaqr_estimate_bytes(const spaqr_symbolic* sym, const spaqr_opts* opts, int64_t nrhs,
                                  size_t* bytes);

#ifdef __cplusplus
}
#endif
#endif /* SPAQR_H */
