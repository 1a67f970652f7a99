/*
 * tridiag_eigvecs: eigenvectors of a real symmetric tridiagonal matrix by
 * inverse iteration with compact-WY re-orthogonalization, on AMD Instinct
 * MI355X (gfx950), FP64 throughout.
 *
 * Method: H. Ishigami, K. Kimura, Y. Nakamura, "On Implementation and
 * Evaluation of Inverse Iteration Algorithm with compact WY Orthogonalization",
 * arXiv:1209.1910.
 *   - Eigenvalues: Sturm-count bisection (the experiments of section 5.1 take
 *     the eigenvalues from bisection).
 *   - Clusters: eigenvalue j joins the cluster of j-1 when
 *     lambda_j - lambda_{j-1} <= 1e-3 ||T||_1 (section 2.1; Alg. 1 and 4).
 *   - Iteration: solve (T - lambda_j I) v^(k) = v^(k-1) (Eq. (1)) after
 *     normalizing v^(k-1), by default a fixed number of times (3);
 *     te_opts.stop selects a growth-based stopping rule instead.
 *   - Within a cluster, each iterate is re-orthogonalized against the previous
 *     members with the compact WY representation, Eqs. (cwy1)-(cwy2), in the
 *     form of section 3.3.2, as Alg. 4 prescribes.
 *
 * Conventions for every entry point:
 *   - T = tridiag(e, d, e): d has n entries, e has n - 1.
 *   - Pointers named d, e, W, Z, d_all, ... are DEVICE pointers to memory the
 *     caller allocated and owns; the library never frees or retains them after
 *     the work it enqueued has completed.
 *   - Work runs on `stream` (a hipStream_t; 0 is the null stream).  Between
 *     the cluster detection and the cluster chains every eigenvector entry
 *     point copies the cluster table to the host to plan the chains, and it
 *     synchronizes `stream` before returning: on return the outputs are ready.
 *   - Index ranges are LAPACK style: 1 <= il <= iu <= n, inclusive; m = iu - il + 1.
 *   - Outputs: W[0..m-1] ascending eigenvalues lambda_il..lambda_iu; column j of
 *     Z (column-major, leading dimension ldz >= n) is the unit-2-norm
 *     eigenvector of W[j], its largest-magnitude entry (lowest index on ties)
 *     made positive.
 *   - Return value: 0 on success; -i when argument i (1-based) is invalid,
 *     detected on the host before anything is enqueued; TE_ERR_* below on a
 *     runtime failure (the HIP error is available from te_last_hip_error()).
 *
 * Start vectors: entry i of v^(0) for eigenvalue index k (1-based, global) is
 * 2u - 1, u = (z >> 11) * 2^-53, z the (((k << 32) | i) + 1)-th output of the
 * SplitMix64 stream seeded with `seed` (Steele, Lea, Flood, OOPSLA 2014).  The
 * plain entry points use TE_DEFAULT_SEED.  Keying by the global index makes a
 * range request compute, for every cluster fully inside the range, exactly the
 * vectors of the full request.
 */
#ifndef TRIDIAG_EIGVECS_H
#define TRIDIAG_EIGVECS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TE_DEFAULT_SEED 0x12091910ULL
#define TE_DEFAULT_ITERS 3

/* Runtime failures (argument errors are the negative argument position). */
#define TE_ERR_HIP (-1000)        /* a HIP runtime call failed                   */
#define TE_ERR_NO_DEVICE (-1001)  /* no usable gfx950 device                     */
#define TE_ERR_WORKSPACE (-1002)  /* workspace too small / allocation failed     */
#define TE_ERR_KERNEL (-1003)     /* a cooperative chain barrier timed out       */
#define TE_ERR_UNSUPPORTED (-1004) /* the options do not apply to this input:
                                      orth = TE_ORTH_MGS with n > TE_MGS_MAX_N   */

/* Per-vector status bits (info[1 + j] of the _ex and _noalloc entry points).
 * TE_INFO_NONFINITE: the vector has a non-finite entry (or is zero).
 * TE_INFO_BREAKDOWN: in one of its compact-WY steps the rows of Q^T v from
 *   the member's own row down were exactly zero (||u_hat|| = 0 in Eq. (yt)):
 *   no reflector exists, H = I and t = 0 are used, and the iterate becomes the
 *   next column of the accumulated orthogonal matrix.
 * TE_INFO_PIVOT: a pivot of the LU of T - lambda_j I (partial pivoting) was
 *   below eps ||T||_1 in magnitude and was replaced by +-eps ||T||_1; common
 *   and harmless when lambda_j is accurate to a few ulps (the solve is then
 *   that of a matrix eps ||T||_1 away).
 * TE_INFO_NOCONV: see TE_STOP_GROWTH. */
#define TE_INFO_NONFINITE 1
#define TE_INFO_BREAKDOWN 2
#define TE_INFO_PIVOT 4
#define TE_INFO_NOCONV 8    /* TE_STOP_GROWTH: no solve of the vector converged */

/* Re-orthogonalization inside a cluster (te_opts.orth).
 * TE_ORTH_CWY: compact WY, the paper's method (Alg. 4 with section 3.3.2).
 * TE_ORTH_MGS: modified Gram-Schmidt against the earlier members' unit
 *   vectors after every solve, the DSTEIN scheme the paper starts from and
 *   compares against (Alg. 1).  Each chain runs in one workgroup with the
 *   iterate in registers, so it takes problems of order n <= TE_MGS_MAX_N. */
#define TE_ORTH_CWY 0
#define TE_ORTH_MGS 1
#define TE_MGS_MAX_N 8192

/* Stop test of the repeat loop (te_opts.stop).  Alg. 1 and Alg. 4 repeat
 * "until some condition is met" without naming it.
 * TE_STOP_FIXED: a fixed number of iterations, te_opts.iters (default 3).
 * TE_STOP_GROWTH: in the manner of the inverse-iteration code the paper
 *   starts from: a solve (T - lambda I) x = v with ||v||_2 = 1 has converged
 *   when ||x||_2 >= 1 / (n eps ||T||_1) (1/||x||_2 is the residual of
 *   x/||x||_2; ||x||^2 summed from the last row up); the first converged
 *   solve is followed by 2 more iterations, 5 at most.  A vector none of
 *   whose solves converged gets TE_INFO_NOCONV. */
#define TE_STOP_FIXED 0
#define TE_STOP_GROWTH 1

/* Options for the _ex entry point.  Zero-initialize and set what you need;
 * a zero field means the default. */
typedef struct te_opts {
    int iters;          /* inverse-iteration steps per vector (default 3)          */
    int orth;           /* TE_ORTH_CWY (default) or TE_ORTH_MGS                     */
    uint64_t seed;      /* start-vector seed (default TE_DEFAULT_SEED)              */
    double cluster_rtol;/* cluster gap as a multiple of ||T||_1 (default 1e-3)      */
    int coop_wgs;       /* cap on cooperative workgroups (0: fill the device)       */
    int stop;           /* TE_STOP_FIXED (default): `iters` iterations per vector;
                           TE_STOP_GROWTH: the growth rule below (iters unused)     */
    uint64_t ws_budget; /* device workspace budget in bytes for batched calls
                           (0: half the free device memory, at most 64 GiB)         */
} te_opts;

/* Eigenpairs il..iu of T (bisection for W, then inverse iteration).
 * Argument positions for error codes: d=1 e=2 n=3 il=4 iu=5 W=6 Z=7 ldz=8.
 * Allocates its workspace with hipMallocAsync on `stream` and frees it before
 * returning (the memory pool may keep it cached). */
int tridiag_eigvecs(const double *d, const double *e, int n, int il, int iu,
                    double *W, double *Z, int ldz, hipStream_t stream);

/* Eigenvectors for m caller-supplied eigenvalue approximations W[0..m-1]
 * (ascending, device memory), the role the paper's DSTEIN-cWY plays after
 * bisection (section 4).  Start vectors are keyed by k = j + 1.
 * Argument positions: d=1 e=2 n=3 m=4 W=5 Z=6 ldz=7. */
int tridiag_eigvecs_given_w(const double *d, const double *e, int n, int m,
                            const double *W, double *Z, int ldz, hipStream_t stream);

/* Upper bound, in bytes, of the device workspace the _ex entry point needs for
 * one problem of order n with indices il..iu.  Returns 0 for invalid sizes. */
size_t tridiag_eigvecs_workspace_bytes(int n, int il, int iu);

/* As tridiag_eigvecs with options and a caller-provided device workspace `ws`
 * of at least tridiag_eigvecs_workspace_bytes(n, il, iu) bytes (256-byte
 * aligned).  If W_given is non-NULL the eigenvalues are taken from it (device,
 * m entries, ascending) and copied to W instead of bisecting.  info (device,
 * may be NULL) receives 1 + m ints: info[1 + j] the TE_INFO_* status bits of
 * vector j, info[0] the number of vectors with any bit set.
 * Argument positions: d=1 e=2 n=3 il=4 iu=5 W_given=6 W=7 Z=8 ldz=9 opt=10
 * ws=11 ws_bytes=12 info=13. */
int tridiag_eigvecs_ex(const double *d, const double *e, int n, int il, int iu,
                       const double *W_given, double *W, double *Z, int ldz,
                       const te_opts *opt, void *ws, size_t ws_bytes, int *info,
                       hipStream_t stream);

/* Eigenpairs il..iu of T split into unreduced blocks.  The paper does not
 * split; the bisection and inverse-iteration codes its method builds on work
 * block by block (section 4, section 5.1).  e_i is negligible when
 * e_i^2 <= eps^2 |d_i d_{i+1}| + DBL_MIN; T is then the direct sum of its
 * unreduced blocks and each block is an independent problem (its own norm,
 * cluster gap and pivot floor), so clusters never span blocks.  The
 * eigenvalues of all blocks in ascending order (ties: lower block first) are
 * numbered 1..n and il..iu select from that order; W[j] and column j of Z are
 * the j-th selected eigenpair, the vector exactly zero outside its block.
 * Eigenvalue l (0-based, ascending) of the block that starts at row s uses
 * start-vector key s + 1 + l (rows counted within the block); without a
 * negligible e_i the result is that of tridiag_eigvecs_ex bit for bit.
 * opt as for tridiag_eigvecs_ex (may be NULL).  info (device, may be NULL):
 * 1 + m ints as for tridiag_eigvecs_ex.  nblocks (host, may be NULL)
 * receives the number of blocks.  Allocates its workspace with
 * hipMallocAsync on `stream` and synchronizes `stream` before returning.
 * Argument positions: d=1 e=2 n=3 il=4 iu=5 W=6 Z=7 ldz=8 opt=9. */
int tridiag_eigvecs_split(const double *d, const double *e, int n, int il, int iu, double *W,
                          double *Z, int ldz, const te_opts *opt, int *info, int *nblocks,
                          hipStream_t stream);

/* Singular values and vectors of an upper bidiagonal matrix B (diagonal a[0..n-1],
 * superdiagonal b[0..n-2], device arrays), the application the paper names
 * for its method (section 6).  B's Golub-Kahan tridiagonal of order 2n (zero
 * diagonal, off-diagonal a_0, b_0, a_1, ..., b_{n-2}, a_{n-1}) has eigenvalues
 * +-sigma_i, and an eigenvector (x_0, y_0, x_1, y_1, ...) of +sigma gives
 * B x = sigma y, B^T y = sigma x.  The singular values in ascending order,
 * indices il..iu of 1..n, are that tridiagonal's eigenvalues n + il .. n + iu,
 * computed with the same method (bisection, clusters among the requested
 * ones, inverse iteration with compact-WY re-orthogonalization, start-vector
 * keys n + il + j).  S[j] receives sigma, column j of V (ld ldv) the x half and
 * column j of U (ld ldu) the y half of its vector, each normalized to unit
 * 2-norm.  A singular value below half the cluster gap (1e-3 of the
 * tridiagonal's 1-norm) shares a cluster with its negative, which is not
 * requested: the two halves are then normalized separately, which keeps their
 * directions.  info (device, may be
 * NULL): 1 + m status ints as for tridiag_eigvecs_ex.  Allocates its
 * workspace with hipMallocAsync and synchronizes `stream` before returning.
 * Argument positions: a=1 b=2 n=3 il=4 iu=5 S=6 U=7 ldu=8 V=9 ldv=10 opt=11. */
int bidiag_svd(const double *a, const double *b, int n, int il, int iu, double *S, double *U,
               int ldu, double *V, int ldv, const te_opts *opt, int *info, hipStream_t stream);

/* ---- Entry point that allocates nothing ----
 * For callers that cannot allocate device memory while they run: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same method, arguments and results as tridiag_eigvecs_ex (bit-identical),
 * without the workspace arguments: the workspace is a fixed device array of
 * TE_NOALLOC_SCRATCH_BYTES inside the library, one per device, held from the
 * first call on that device until the process ends.  No device memory is
 * allocated or freed by the call (host-side planning uses small host
 * vectors).  Problems whose workspace (tridiag_eigvecs_noalloc_bytes) exceeds
 * TE_NOALLOC_SCRATCH_BYTES are rejected with TE_ERR_WORKSPACE before anything
 * is enqueued.  Every call on a device shares that device's array: calls
 * that overlap in time on one device (several host threads or streams) race
 * and must be serialized by the caller; a call that has returned has finished
 * with it (the entry point synchronizes `stream`).
 * Argument positions: d=1 e=2 n=3 il=4 iu=5 W_given=6 W=7 Z=8 ldz=9 opt=10
 * info=11. */
#define TE_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

int tridiag_eigvecs_noalloc(const double *d, const double *e, int n, int il, int iu,
                            const double *W_given, double *W, double *Z, int ldz,
                            const te_opts *opt, int *info, hipStream_t stream);

/* Workspace bytes tridiag_eigvecs_noalloc needs for one problem (0 for invalid
 * sizes); the call accepts the problem when this is at most
 * TE_NOALLOC_SCRATCH_BYTES. */
size_t tridiag_eigvecs_noalloc_bytes(int n, int il, int iu);

/* B independent problems, processed together.  Problem b has order
 * n_b = off[b+1] - off[b]; its d entries are d_all[off[b] .. off[b+1]-1] and
 * its e entries e_all[off[b] - b .. off[b+1] - b - 2] (n_b - 1 of them).
 * il[b], iu[b] (host arrays) select its eigenvalues; W_all[woff[b] ..] receives
 * them and Z_all + zoff[b] its eigenvectors with leading dimension n_b, where
 * woff/zoff (host arrays of B entries) are caller-chosen offsets.  off, il, iu,
 * woff, zoff are HOST arrays; d_all, e_all, W_all, Z_all are device arrays.
 * Consecutive problems are grouped into sub-batches whose workspace fits
 * opt->ws_budget; each sub-batch runs every phase as one launch over all of
 * its problems (their cluster chains run concurrently).  Synchronizes
 * `stream` before returning.  Returns TE_ERR_WORKSPACE if a single problem
 * does not fit the budget.
 * Argument positions: d_all=1 e_all=2 off=3 il=4 iu=5 W_all=6 woff=7 Z_all=8
 * zoff=9 B=10 opt=11. */
int tridiag_eigvecs_batched(const double *d_all, const double *e_all, const int64_t *off,
                            const int *il, const int *iu, double *W_all, const int64_t *woff,
                            double *Z_all, const int64_t *zoff, int B, const te_opts *opt,
                            hipStream_t stream);

/* tridiag_eigvecs_batched with per-vector status words.  Arguments 1-11 and
 * their error positions as for tridiag_eigvecs_batched.  info_all (device)
 * receives, for problem b, 1 + m_b ints at info_all + ioff[b] (m_b =
 * iu[b] - il[b] + 1) laid out as the info of tridiag_eigvecs_ex: entry 1 + j
 * the TE_INFO_* bits of the problem's vector j, entry 0 how many of its
 * vectors have any bit set.  ioff (host, B entries) are caller-chosen offsets;
 * the B regions must not overlap (else -13).  Results other than info are
 * those of tridiag_eigvecs_batched.
 * Argument positions: 1-11 as above, info_all=12 ioff=13. */
int tridiag_eigvecs_batched_ex(const double *d_all, const double *e_all, const int64_t *off,
                               const int *il, const int *iu, double *W_all, const int64_t *woff,
                               double *Z_all, const int64_t *zoff, int B, const te_opts *opt,
                               int *info_all, const int64_t *ioff, hipStream_t stream);

/* ---- Graph-captured batched path ----
 * The batched method with every step on the device, captured once into a
 * hipGraph and then run by one graph launch per call.  The chain plan that
 * tridiag_eigvecs_batched makes on the host (after reading the cluster tables
 * back) is made here by device kernels: every cluster of two or more members
 * becomes a chain, ordered by decreasing cost size^2 n, and a persistent
 * kernel runs each chain in one workgroup.  Results are bit-identical to
 * tridiag_eigvecs_batched and to tridiag_eigvecs problem by problem (the
 * chains' sums have one fixed order whatever the workgroup size).  Since a
 * chain never spreads over several workgroups here, this path suits batches of
 * many moderate problems (the cooperative multi-workgroup chain of the other
 * entry points is not used).  With orth = TE_ORTH_MGS the chains run the MGS
 * kernel (one workgroup of 512 threads per chain, as in the other entry
 * points; problems of order n <= TE_MGS_MAX_N, else TE_ERR_UNSUPPORTED), with
 * results bit-identical to tridiag_eigvecs_batched under the same options.
 * te_batch_autotune tunes the compact-WY chain only (TE_ERR_UNSUPPORTED for
 * MGS options). */

/* Launch configuration of the chain kernel of the graph path.
 * chain_threads: threads per chain workgroup (256 or 512).
 * chains_per_cu: resident chain workgroups per compute unit (1 .. the
 * occupancy limit of that variant). */
typedef struct te_graph_cfg {
    int chain_threads;
    int chains_per_cu;
} te_graph_cfg;

typedef struct te_batch_graph te_batch_graph;

/* Build the graph for B problems laid out as for tridiag_eigvecs_batched (same
 * arguments 1-11 with the same meaning and error positions).  The device
 * pointers d_all, e_all, W_all, Z_all are captured: every launch reads the
 * inputs they hold at that time and writes the outputs there.  cfg (argument
 * 12) may be NULL: then the autotune table's entry for this batch's shape
 * (see te_batch_autotune) is used, else {256, the occupancy limit}; for MGS
 * options {512, the MGS kernel's occupancy limit} (a given cfg must have
 * chain_threads = 512 there).
 * Problems are grouped into consecutive segments whose workspace fits
 * opt->ws_budget (default: half the free device memory, at most 64 GiB); the
 * segments run one after another inside the graph and share one workspace.
 * The graph owns its device memory (hipMalloc at creation; see
 * te_batch_graph_info) until te_batch_graph_destroy.  Returns NULL on failure
 * with *rc (may be NULL) set to the error code (TE_ERR_WORKSPACE if a single
 * problem does not fit the budget or the memory cannot be allocated). */
te_batch_graph *te_batch_graph_create(const double *d_all, const double *e_all, const int64_t *off,
                                      const int *il, const int *iu, double *W_all,
                                      const int64_t *woff, double *Z_all, const int64_t *zoff,
                                      int B, const te_opts *opt, const te_graph_cfg *cfg,
                                      int *rc);

/* Run the whole batch: one hipGraphLaunch on `stream`, which is synchronized
 * before returning.  Call on the device the graph was built on.
 * Returns 0, -1 for a NULL graph, TE_ERR_KERNEL if a chain's internal wait
 * timed out (its results are then incomplete), or another TE_ERR_*. */
int te_batch_graph_launch(te_batch_graph *g, hipStream_t stream);

/* The graph's chain configuration, number of segments and device bytes it
 * owns (any pointer may be NULL).  Returns 0, or -1 for a NULL graph. */
int te_batch_graph_info(const te_batch_graph *g, te_graph_cfg *cfg, int *segments,
                        uint64_t *device_bytes);

/* Free the graph and its device memory (waits for the device). */
void te_batch_graph_destroy(te_batch_graph *g);

/* Autotuner of the graph path.  Times every candidate configuration
 * (chain_threads 256 and 512, chains_per_cu 1, 2, 4, ... up to each variant's
 * occupancy limit) on a sample of the batch (every (B / 2048)-th problem,
 * every problem when B < 4096): one warm-up launch and one timed launch
 * of that sample's graph each.  The fastest goes into the process's autotune
 * table under the batch's shape key (ceil log2 of the largest n, ceil log2 of
 * the mean n), and, when the environment variable TE_TUNE_FILE names a file,
 * is appended to it as a line "nbits mbits chain_threads chains_per_cu"; that
 * file is read once, on first use of the table.  The sampled problems'
 * results are written to W_all and Z_all.  best (may be NULL) receives the
 * winner; tried and ms (may be NULL, cap entries) the candidates and their
 * times in milliseconds, *ntried (may be NULL) how many were timed.
 * Arguments 1-11 as for te_batch_graph_create. */
int te_batch_autotune(const double *d_all, const double *e_all, const int64_t *off, const int *il,
                      const int *iu, double *W_all, const int64_t *woff, double *Z_all,
                      const int64_t *zoff, int B, const te_opts *opt, te_graph_cfg *best,
                      te_graph_cfg *tried, double *ms, int cap, int *ntried);

/* Eigenvalues only: lambda_il..lambda_iu of T by Sturm-count bisection, into
 * W[0..m-1] (device).  Counts are exact integers; W is the bracket midpoint
 * after the bracket [gl, gu] (Gershgorin, widened until count(gl) = 0 and
 * count(gu) = n) has been halved until it is at most 2 eps max(|gl|,|gu|)
 * wide.  Synchronizes `stream` before returning.
 * Argument positions: d=1 e=2 n=3 il=4 iu=5 W=6. */
int tridiag_eigvals(const double *d, const double *e, int n, int il, int iu, double *W,
                    hipStream_t stream);

/* Peters-Wilkinson clusters of m ascending values W (device): j starts a new
 * cluster iff j = 0 or W[j] - W[j-1] > tol (section 2.1; Alg. 1 and 4).
 * Writes the cluster starts and sizes (device int arrays of at least m
 * entries) and their count *ncl (device int).  Synchronizes `stream`.
 * Argument positions: W=1 m=2 tol=3 start=4 size=5 ncl=6. */
int tridiag_clusters(const double *W, int m, double tol, int *start, int *size, int *ncl,
                     hipStream_t stream);

/* ---- Serving engine ----
 * A request loop for eigenvector solves of different sizes arriving over
 * time (continuous batching; the method and its results are those of
 * tridiag_eigvecs, problem by problem, bit for bit).  Requests wait in two
 * FIFO queues, light and heavy, by the size of their per-eigenvalue state
 * (n * m below or at least 2^22 entries).  Each of `lanes` host threads owns a
 * stream; a free lane takes the class of the oldest waiting request and
 * admits from that queue, in order, every request whose device memory (its
 * inputs, outputs and workspace) still fits the HBM budget beside the rounds
 * in flight, up to 512.  The round then runs every phase as one launch over
 * its requests, copies W and Z to the caller's buffers and frees its memory;
 * rounds on different lanes overlap on the device.  A request whose own need
 * exceeds the budget completes at once with TE_ERR_WORKSPACE.
 * Memory from the round's device allocations stays cached in the device's
 * stream-ordered pool after use, so the process's device footprint can exceed
 * the budget by the pool's fragmentation.
 * All functions are thread-safe. */
typedef struct te_server te_server;

/* Start a server on the current device.  hbm_budget: device bytes that
 * admitted requests may hold at once (0: half the free device memory, at most
 * 64 GiB).  lanes: concurrent rounds (0: 3; at most 64).  opt: as for
 * tridiag_eigvecs_ex (may be NULL); coop_wgs = 0 lets the cooperative chain
 * kernel fill the device (a smaller cap leaves compute units to the other
 * lanes while it runs, at the cost of its own speed).  Returns NULL if there
 * is no usable device or an argument is invalid. */
te_server *te_server_create(uint64_t hbm_budget, int lanes, const te_opts *opt);

/* Queue one request: eigenpairs il..iu of T = tridiag(e, d, e) of order n.
 * d (n) and e (n - 1) are HOST arrays, copied before the call returns.  W (m
 * doubles) and Z (column-major, leading dimension ldz >= n, m columns) are
 * host or device memory that receive the results when the request completes;
 * they must stay valid until then.  *id receives the request id.
 * Argument positions: server=1 d=2 e=3 n=4 il=5 iu=6 W=7 Z=8 ldz=9 id=10;
 * TE_ERR_NO_DEVICE if the server is shutting down. */
int te_server_submit(te_server *server, const double *d, const double *e, int n, int il, int iu,
                     double *W, double *Z, int ldz, int64_t *id);

/* 1 if request id has completed (then *rc, if rc is non-NULL, is its result
 * code, 0 or a TE_ERR_* value), 0 if it is still queued or running, -1 for a
 * NULL server, -2 for an unknown id. */
int te_server_poll(te_server *server, int64_t id, int *rc);

/* Block until request id has completed; returns as te_server_poll. */
int te_server_wait(te_server *server, int64_t id, int *rc);

/* Seconds since te_server_create at which request id was submitted, admitted
 * into a round and completed (results in the caller's buffers).  Any pointer
 * may be NULL.  Returns as te_server_poll. */
int te_server_times(te_server *server, int64_t id, double *t_submit, double *t_start,
                    double *t_done);

/* Forget a completed request: the server frees its record (status and
 * times), after which its id is unknown to poll, wait and times.  A server
 * keeps every request's record until it is released or the server is
 * destroyed, so a long-running caller releases each request once it has read
 * what it needs.  Returns 1 when released, 0 if the request has not completed
 * yet (nothing is changed), -1 for a NULL server, -2 for an unknown id. */
int te_server_release(te_server *server, int64_t id);

/* Finish every queued request, stop the lanes and free the server. */
void te_server_destroy(te_server *server);

/* Device-time accounting of the library's kernels, for benchmarks and
 * profiling.  When enabled, every entry point records hipEvents around each
 * kernel it launches, on the stream it launches it on, and adds the elapsed
 * milliseconds to per-phase totals (process-wide, guarded by a mutex).
 * Phases: 0 setup, 1 bisection, 2 clusters, 3 first solves (one lane per
 * eigenvalue), 4 transpose, 5 small cluster chains, 6 cooperative cluster
 * chains, 7 finalize.  te_timing_read copies min(cap, 8) totals and launch
 * counts (either pointer may be NULL) and returns 8. */
void te_timing_enable(int on);
void te_timing_reset(void);
int te_timing_read(double *ms, long long *launches, int cap);

/* HIP error code of the last runtime failure seen by this thread (0 if none). */
int te_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TRIDIAG_EIGVECS_H */
