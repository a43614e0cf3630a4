/*
 * grest.h -- C interface of libgrest, the MI355X (gfx950) implementation of the
 * G-REST eigenpair update for evolving graphs.
 *
 * Method (Eini, Karaaslanli, Kalantzis, Traganitis, "Subspace Projection Methods
 * for Fast Spectral Embeddings of Evolving Graphs"):
 *   - transition model, Sec. 2 eq. (adj_update): A^(t+1) = pad(A^(t)) + Delta with
 *     Delta = [[K, G], [G^T, C]] (edge flips among old nodes, edges of appended nodes);
 *   - single-step problem, Sec. 2.1 (Problem 1): given K eigenpairs of A and Delta,
 *     estimate K eigenpairs of A^(t+1);
 *   - tracking loop, Alg. 2: pad X, build an orthonormal basis Z of
 *     [Xbar, (I - Xbar Xbar^T)[Delta Xbar, B2]] (Sec. 3.3, Table 1) with
 *     B2 = Delta_2 (G-REST3), B2 = the rank-L randomized basis R of Sec. 3.5
 *     (G-REST_RSVD), or no B2 (G-REST2), then Rayleigh-Ritz (Alg. 1) on
 *     Z^T A^(t+1) Z (eq. RR_eigen_graph_upd_main2) and X <- Z F_K;
 *   - shifted Laplacians, Sec. 4.2: the trailing pairs of L = D - A and of
 *     L_n = I - D^{-1/2} A D^{-1/2} are the leading pairs of alpha I - L and 2 I - L_n.
 *
 * Groups of entry points: a state's life (create, set or init pairs, update, sync,
 * get, shape, destroy); the truncated projection of eq. RR_eigen_graph_upd_main3 with a
 * released graph (GREST_PROJ_LOWRANK, grest_release_graph); drift and recomputation
 * (grest_drift, grest_set_restart); checkpoint, resume and the borrowed view (grest_save,
 * grest_load, grest_view); streams, overlap, memory and stage timing; and the server
 * that runs many graphs' updates together (grest_server_*, grest_submit, grest_poll).
 *
 * Conventions shared by every entry point:
 *   - All functions return a grest_status; no exception crosses the interface.
 *   - Node ids are int32 (graphs below 2^31 nodes); each undirected edge change is
 *     given once as (i, j) with i < j and a sign +1 (insert) or -1 (delete).  An edge
 *     that touches an appended node (id >= current node count) is an insertion.
 *   - Dense blocks are row-major.  "Host" pointers are ordinary CPU memory, "device"
 *     pointers are HIP device memory on the state's device.
 *   - The caller owns every buffer it passes; the library copies inputs before the
 *     call returns (host inputs) or before the work that reads them is finished on
 *     the state's stream (device inputs: keep them alive until grest_sync).
 *   - A state is driven from one host thread at a time; different states are
 *     independent.
 */
#ifndef GREST_H
#define GREST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct grest_state grest_state;

typedef enum grest_status {
  GREST_OK = 0,
  GREST_EINVAL = 1,   /* bad argument, or a change list that breaks the transition model */
  GREST_ENOMEM = 2,   /* device or host allocation failed */
  GREST_EDEVICE = 3,  /* HIP runtime error (see grest_last_error) */
  GREST_ENUMERIC = 4, /* non-finite value or eigensolver without convergence */
  GREST_ENODEV = 5,   /* no usable device */
  GREST_EAGAIN = 6    /* server queue full or device-memory budget exceeded; retry later */
} grest_status;

/* operator whose pairs are tracked (Sec. 4.2) */
enum { GREST_OP_ADJ = 0, GREST_OP_LAP = 1, GREST_OP_NLAP = 2 };
/* subspace (Table 1, Sec. 3.5) */
enum { GREST_G2 = 2, GREST_G3 = 3, GREST_RSVD = 4 };
/* arithmetic of the dense blocks: all FP64; FP32 blocks with FP64 Gram/Cholesky/eigensolve;
 * FP32 blocks with BF16-MFMA products Z^T(AZ) and Z F (FP32 accumulation) */
enum { GREST_FP64 = 0, GREST_FP32 = 1, GREST_MIXED = 2 };
/* where a pointer lives */
enum { GREST_HOST = 0, GREST_DEVICE = 1 };
/* element type of a dense output */
enum { GREST_F64 = 0, GREST_F32 = 1 };
/* projected matrix of the Rayleigh-Ritz step: EXACT, H = Z^T A' Z with the stored updated
 * graph (eq. RR_eigen_graph_upd_main2); LOWRANK, H = Z^T (Xbar Theta Xbar^T + Delta) Z
 * with the previous Ritz values Theta (eq. RR_eigen_graph_upd_main3, the form of Alg. 2),
 * which needs no product with the whole graph (adjacency and combinatorial Laplacian: for
 * T = alpha I - L the change of T is Delta minus the degree changes on the rows of Delta,
 * plus (alpha' - alpha) I on the old nodes and alpha' I on the appended ones) */
enum { GREST_PROJ_EXACT = 0, GREST_PROJ_LOWRANK = 1 };

typedef struct grest_config {
  int32_t k;          /* K, number of tracked pairs (>= 1) */
  int32_t variant;    /* GREST_G2 / GREST_G3 / GREST_RSVD */
  int32_t L;          /* RSVD rank L (variant RSVD) */
  int32_t P;          /* RSVD oversampling P (variant RSVD) */
  int32_t op;         /* GREST_OP_* */
  int32_t precision;  /* GREST_FP64 / GREST_FP32 / GREST_MIXED */
  int32_t max_new;    /* largest S per update for G-REST3 (sizes the basis block) */
  int32_t proj;       /* GREST_PROJ_EXACT (0) or GREST_PROJ_LOWRANK (op ADJ or LAP) */
  double rank_tol;    /* relative rank threshold of the orthonormalisation; 0 = default
                         (1e-7 in FP64, 1e-5 otherwise) */
} grest_config;

/* ABI version of this header (bumped on any incompatible change). */
int32_t grest_abi_version(void);

/* Message of a status code (static string). */
const char* grest_strerror(grest_status status);

/* Text of the last HIP error seen by this thread (static thread-local buffer). */
const char* grest_last_error(void);

/*
 * Format check of a change list on the host, without a device: ids in range,
 * i < j, sign +1/-1, edges of appended nodes are insertions, no pair twice.
 * n: current node count, n_new: appended nodes S.  Host pointers.
 * Returns GREST_OK or GREST_EINVAL.  (Membership -- insert of an existing edge,
 * delete of a missing one -- needs the stored graph and is checked by grest_update.)
 */
grest_status grest_validate_changes(int64_t n, int64_t n_new, int64_t n_changes, const int32_t* ei,
                                    const int32_t* ej, const int8_t* sign);

/*
 * Create a state for the graph A^(0) (Sec. 2; Alg. 2 input), stored on the current
 * HIP device.  rowptr (n0+1 entries, int64) and col (rowptr[n0] entries, int32) are
 * host pointers to a symmetric CSR with both triangles, sorted columns, no self-loops
 * and no duplicates (checked: GREST_EINVAL).  node_capacity / nnz_capacity reserve
 * room for growth (0 = automatic; buffers grow on demand with a device
 * synchronisation).  The change-list buffers start sized for a change list of 1/32 of
 * the stored entries (4,096 changes for a low-rank state) and the sketch buffers for
 * n0/64 appended nodes; they too grow on demand.  stream: a hipStream_t of that device, or NULL for a private
 * stream.  The tracked pairs are unset until grest_set_pairs or grest_init_pairs.
 * Widths: 1 <= k <= 128 and k < n0; the basis width D = k + Dw with Dw = k (G-REST2),
 * k + max_new (G-REST3) or k + L (RSVD) is at most 196; every block orthonormalised by
 * CholQR2 is at most 128 wide (G-REST2/3: Dw; RSVD: k and L + P).  Node counts and
 * node_capacity stay below 2^31 - 1 (node ids are int32).  Otherwise GREST_EINVAL.
 */
grest_status grest_create(const grest_config* cfg, void* stream, int64_t n0, const int64_t* rowptr,
                          const int32_t* col, int64_t node_capacity, int64_t nnz_capacity,
                          grest_state** out);

/*
 * Set the tracked pairs (Alg. 2 line 3 computed by the caller): values[k] (adjacency:
 * eigenvalues of A; Laplacians: eigenvalues nu of L or L_n) and X, n x k row-major with
 * orthonormal columns, FP64.  where: GREST_HOST or GREST_DEVICE for both pointers.
 */
grest_status grest_set_pairs(grest_state* st, const double* values, const double* X, int32_t where);

/*
 * Compute initial pairs on the device (Alg. 2 line 3; the paper allows any direct
 * eigendecomposition method): a Chebyshev-filtered block subspace iteration built from the
 * update kernels.  The block has min(width, 128, n) columns (width = the basis width of
 * the state, K + Dw); after a random start orthonormalised by CholQR2, every outer step
 * runs Rayleigh-Ritz on the block (FP64 small eigensolve of all its pairs), measures
 * resid = max_{j < k} ||M x_j - lambda_j x_j||_2 / scale (M and scale as for grest_drift),
 * and, unless resid <= tol or the budget is spent, applies the Chebyshev polynomial of
 * the operator that damps the interval of the unwanted spectrum (its degree bounded so
 * that the filtered block stays well conditioned, at most 16) followed by CholQR2.
 * iterations: largest number of products with the operator (>= 1); seed: start block.
 * grest_init_pairs uses the precision's default tolerance (1e-12 with FP64 blocks, 4e-6
 * otherwise); grest_init_pairs_tol takes tol (>= 0; 0 runs the whole budget) and returns
 * the products used and the final resid (either pointer may be NULL).  The pairs of the
 * last Rayleigh-Ritz step are kept whether or not tol was reached; GREST_ENUMERIC on a
 * non-finite value.  EINVAL on a NULL state, iterations < 1, a negative or NaN tol or a
 * state without its graph.
 */
grest_status grest_init_pairs(grest_state* st, int32_t iterations, uint64_t seed);
grest_status grest_init_pairs_tol(grest_state* st, int32_t max_products, double tol, uint64_t seed,
                                  int32_t* products, double* resid);

/* Products with the operator and final residual of the state's last initial eigensolve
 * (grest_init_pairs, grest_init_pairs_tol or a restart); 0 and -1 before the first.
 * Either pointer may be NULL.  EINVAL on a NULL state. */
grest_status grest_init_stats(const grest_state* st, int32_t* products, double* resid);

/*
 * One G-REST update (Alg. 2 loop body) with n_new appended nodes and n_changes edge
 * changes (ei, ej, sign).  omega: the S x (L+P) Gaussian test matrix of the
 * randomized range finder (Sec. 3.5, step S.1), FP64 row-major; required for
 * variant RSVD when n_new > 0, ignored otherwise.  where: GREST_HOST or GREST_DEVICE
 * for all four arrays.
 * The change list is validated before anything is committed: a violation returns
 * GREST_EINVAL and leaves the state exactly as it was.  One update may change at most
 * 16,384 edges at any one node (a longer row of Delta is refused as a violation).  The rest of the update is
 * queued on the state's stream; numerical trouble is reported by grest_sync.
 */
grest_status grest_update(grest_state* st, int64_t n_new, int64_t n_changes, const int32_t* ei,
                          const int32_t* ej, const int8_t* sign, const double* omega, int32_t where);

/*
 * The same update as grest_update, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): it calls
 * no hipMalloc, hipFree or allocating library routine.  Arguments, validation and results
 * are those of grest_update (bitwise the same results, by the same kernels), except:
 *   - nothing grows: the update must fit the state's current capacities (node count,
 *     stored entries, appended nodes of the sketch, the low-rank gather rows), which
 *     grest_create's node_capacity / nnz_capacity or earlier grest_update calls set;
 *   - n_changes <= 262,144 (2^18).  The buffers sized by the change list (its device
 *     copy, Delta's packed keys and their copy grouped by row, the merge ranks, Delta's
 *     columns and signs) live in one static device array of 20 MiB that every device the library
 *     runs on holds until the process ends;
 *   - the change list's format is checked on the device only (the state is still left
 *     unchanged by a violation, with GREST_EINVAL);
 *   - the restart policy of grest_set_restart is not applied by this call.
 * A size beyond these limits returns GREST_EINVAL (grest_last_error names the limit) with
 * nothing queued.  Every call on one device shares that device's array, which keeps the
 * last call's contents: calls that overlap on one device race, so before a no-allocation
 * update of another state on the same device, wait for the previous one (grest_sync).
 * A state's own successive calls are ordered by its streams and do not race.
 */
grest_status grest_update_noalloc(grest_state* st, int64_t n_new, int64_t n_changes, const int32_t* ei,
                                  const int32_t* ej, const int8_t* sign, const double* omega, int32_t where);

/*
 * Updates of several graphs at once (Alg. 2 loop body for each): items[i] names a state
 * and its update, with the arguments of grest_update.  The updates run in lockstep, each
 * on its own state's stream: the one-workgroup stages of the method (the Cholesky factors
 * of CholQR2, Sec. 3.5 step S.2 and the projection of Sec. 4; the small symmetric
 * eigensolves of Alg. 1 and step S.3) are launched once for all graphs, one workgroup per
 * graph, each reading its graph's arguments from a descriptor array in device memory,
 * instead of once per graph.  Every graph gets exactly the computation of its own
 * grest_update (the same kernels with the same arguments), so its results do not depend
 * on the other members.
 *   - 1 <= count <= GREST_BATCH_MAX; the states must be distinct, on one device, and not
 *     updated by another thread meanwhile.  For the graphs' work to overlap, give the
 *     states streams of their own (the default).
 *   - items[i].status receives that member's grest_update status; the call returns
 *     GREST_OK when every member succeeded, else the first member's failure (the others
 *     are applied or refused as their own statuses say; grest_last_error names the
 *     member).  EINVAL with nothing done for a bad count, a NULL or repeated state.
 * Like grest_update, the call returns once the work is queued; grest_sync each state.
 */
#define GREST_BATCH_MAX 64
typedef struct {
  grest_state* state;
  int64_t n_new, n_changes;
  const int32_t* ei;
  const int32_t* ej;
  const int8_t* sign;
  const double* omega;
  int32_t where;
  int32_t status; /* out */
} grest_batch_item;
grest_status grest_update_batch(grest_batch_item* items, int32_t count);

/* Wait for queued work and return (then clear) deferred numerical status bits. */
grest_status grest_sync(grest_state* st);

/*
 * Copy the tracked pairs out: values[k] (FP64, host; may be NULL), and X (n x k
 * row-major, element type x_dtype, may be NULL) to host or device memory.  Values are
 * ordered as tracked: adjacency by decreasing magnitude, Laplacians by increasing nu.
 */
grest_status grest_get(grest_state* st, double* values, void* X, int32_t x_dtype, int32_t where);

/* Current node count, stored entries (both triangles; -1 once the graph is released)
 * and the state's dimensions.  Any output pointer may be NULL. */
grest_status grest_shape(const grest_state* st, int64_t* n, int64_t* nnz, int32_t* k, int32_t* width);

/*
 * Copy the stored graph to host memory: rowptr (n+1 int64) and col (nnz int32), for
 * checking the graph update bit for bit.  Waits for queued work.  EINVAL on a NULL state
 * or one that released its graph.
 */
grest_status grest_get_graph(grest_state* st, int64_t* rowptr, int32_t* col);

/*
 * Stage timing with HIP events recorded on the state's stream around the stages of
 * every update while enabled: 0 graph update and validation (with its host wait),
 * 1 padding and Delta Xbar, 2 augmentation block, 3 projections and CholQR2,
 * 4 product with the updated operator, 5 projected matrix Z^T (A Z), 6 small
 * eigensolve, 7 back-projection.  grest_profile(st, 1) enables and clears the
 * totals; grest_profile(st, 2) records only the two events around the sparse product
 * (each timing event between two kernels costs the stream a few microseconds; the
 * stage times then read zero); 0 disables; other values: EINVAL.
 * grest_stage_times returns the accumulated milliseconds per stage, the
 * milliseconds of the sparse product kernel alone, the number of updates, and the sum
 * over those updates of the sparse product's width (the columns of Z it multiplied:
 * all of them, or only the new ones when the kept adjacency product A X is reused).
 * Any output pointer may be null.
 */
grest_status grest_profile(grest_state* st, int32_t enable);
grest_status grest_stage_times(grest_state* st, double* stage_ms, int32_t n_stages, double* spmm_ms,
                               int64_t* updates, int64_t* spmm_cols);

/*
 * Checkpoint (Alg. 2's state between two time steps): the configuration, the capacities,
 * the stored graph (unless released), the tracked pairs and the kept adjacency product
 * A X with its refresh age, as one self-contained host buffer.  buf == NULL: *bytes
 * receives the size needed.  Otherwise *bytes is the buffer's size; if it is too small,
 * EINVAL with the size needed in *bytes.  Waits for the queued work.  The restart policy,
 * the overlap mode, the stream and the stage timing are not part of a checkpoint.
 */
grest_status grest_save(grest_state* st, void* buf, size_t* bytes);

/*
 * Resume: a new state on the current HIP device (stream as for grest_create) equal to
 * the one saved, so that its updates give bit for bit the results the saved state would
 * have given.  bytes must be the checkpoint's exact size.  EINVAL on a buffer that is not
 * a checkpoint of this ABI version or is truncated; device errors as for grest_create.
 */
grest_status grest_load(const void* buf, size_t bytes, void* stream, grest_state** out);

/*
 * Borrowed view of the tracked block without a copy: *X is the device address of the
 * basis buffer whose first k columns are X (row-major, leading dimension *ld elements,
 * element type *dtype: GREST_F64 or GREST_F32), *n its rows.  Valid until the next call
 * that changes the state (update, set or init of pairs, destroy); its contents are final
 * after grest_sync, or for work ordered after the update on the state's stream.  Any
 * output pointer may be NULL.  EINVAL on a NULL state or one without pairs.
 */
grest_status grest_view(grest_state* st, const void** X, int64_t* n, int64_t* ld, int32_t* dtype);

/* Release the state and all its device memory. */
void grest_destroy(grest_state* st);

/* Rebinds the state to another HIP stream (NULL: a stream of its own).  Waits for the
 * work already queued on the old stream first.  EINVAL on a NULL state. */
grest_status grest_set_stream(grest_state* st, void* stream);

/*
 * Overlap mode (enable = 1): the graph stage of each update -- the change list turned
 * into Delta's CSR, its validation, the merge into the new CSR (Sec. 2, eq. adj_update)
 * -- runs on a second stream owned by the state, so that it proceeds while the device
 * still finishes the previous update; the rest of the update stays on the state's stream
 * and waits for it with an event.  Results are the same as without it.  Contract: with
 * where = GREST_DEVICE the change arrays given to grest_update must be complete when it
 * is called (the graph stage no longer waits for earlier work of the state's stream);
 * omega is still read on the state's stream.  enable = 0 returns to one stream.  Waits
 * for the queued work first.  EINVAL on a NULL state, EDEVICE if no stream can be made.
 */
grest_status grest_set_overlap(grest_state* st, int32_t enable);

/*
 * Low-rank states only (proj = GREST_PROJ_LOWRANK): release the stored graph.  The
 * low-rank projected matrix needs only Delta and the previous pairs (eq.
 * RR_eigen_graph_upd_main3, Alg. 2), so the state then keeps its basis, Delta and its
 * scratch; the two CSR column buffers and the (op Z) buffer are freed.  Afterwards each
 * update still sorts its change list into Delta's CSR and rejects out-of-range ids, i >= j,
 * signs other than +1/-1 and pairs listed twice, but it can no longer check an insertion
 * against an existing edge or a deletion against a missing one: the caller vouches for
 * those (the results of an update that breaks them are undefined, not an error).
 * grest_init_pairs and grest_get_graph then return EINVAL and grest_shape reports nnz = -1.
 * Waits for the queued work first.  EINVAL on a NULL state, one with the exact
 * projection, a Laplacian state (its shift 2 d_max comes from the stored graph) or one with
 * a restart policy; calling it again is a no-op.
 */
grest_status grest_release_graph(grest_state* st);

/*
 * Drift of the tracked pairs, the measure a restart is decided on (the recomputation of
 * TIMERS when its accumulated error grows, Sec. 2.2): orth = max_ij |(U^T U - I)_ij| and
 * resid = max_j ||M u_j - lambda_j u_j||_2 / scale, where M is the matrix whose values
 * are reported (A, L or L_n) and scale = max_j |lambda_j| for the adjacency, 2 d_max for
 * L and 2 for L_n (bounds on their norms, Sec. 4.2).  Computed on the device now (one
 * product with the graph and two Gram passes, FP64 accumulation); waits for queued work.
 * resid is NaN for a state without its graph.  Either pointer may be NULL.  EINVAL on a
 * NULL state or one without pairs.
 */
grest_status grest_drift(grest_state* st, double* orth, double* resid);

/*
 * Restart policy: after every check_every-th update (0 disables) the drift is measured
 * (that call of grest_update then waits for the update); when resid > tol_resid or
 * orth > tol_orth, and at least min_gap updates have passed since the pairs were last
 * set, initialised or recomputed (Sec. 5 keeps at least 5 updates between
 * recomputations), the pairs are recomputed from scratch by grest_init_pairs with the
 * given iterations and seed + (number of restarts so far).  A restart inside grest_update
 * returns that call's status.  EINVAL on a NULL state, negative counts, iterations < 1
 * or a negative or NaN tolerance when enabled, or a state without its graph.
 */
grest_status grest_set_restart(grest_state* st, double tol_resid, double tol_orth, int32_t check_every,
                               int32_t min_gap, int32_t iterations, uint64_t seed);

/* Restarts so far and the last drift measured by the policy (-1 before the first);
 * any pointer may be NULL. */
grest_status grest_restart_stats(const grest_state* st, int64_t* restarts, double* last_orth, double* last_resid);

/* Device memory held by the state, in bytes (its current capacities). */
grest_status grest_memory(const grest_state* st, int64_t* device_bytes);

/* ------------------------------------------------------------------------------------
 * Batched execution of many graphs (serving).  This is not part of the method: it runs
 * the single-graph update of Alg. 2 for many independent graphs on one device.
 *
 * A server owns `lanes` worker lanes, each a host thread with its own HIP stream.
 * Requests wait in one queue in submission order; a free lane takes the oldest request
 * whose graph no other lane is updating and runs it on its own stream (the graph's state
 * is moved there while idle).  So the updates of one graph run in submission order and
 * one at a time, a request never waits behind another graph's update while a lane is
 * free, and lanes overlap on the device.  Every update of a graph runs the same kernels with the
 * same reduction orders whatever else is queued, so its result does not depend on the
 * mix of graphs.
 *
 * Admission by device memory (hbm_budget_bytes, 0: no limit): the server reserves for
 * every attached graph its current footprint (grest_memory) plus the growth its queued
 * requests will cause (an update that outgrows a capacity reallocates it: node and entry
 * buffers by 1.5x, change and sketch buffers by 2x).  attach fails with GREST_EAGAIN when
 * the state's footprint does not fit the budget; submit fails with GREST_EAGAIN when the
 * request's growth does not fit, or when `max_queue` requests are pending.  Memory frees
 * up when a graph is detached, and when a graph's requests have all run (its reservation
 * is then replaced by its actual footprint); a refused submission can be retried then.
 * Time stamps are nanoseconds of the monotonic clock that grest_now_ns reads.
 * While attached, a state must not be used directly (no update, get or sync) except
 * after grest_server_drain has returned; the server restores the state's original
 * stream when it is destroyed.  Requests for one graph are submitted from one host
 * thread (their order is the submission order).
 * ------------------------------------------------------------------------------------ */
typedef struct grest_server grest_server;

int64_t grest_now_ns(void);

/* lanes in [1, 64]; max_queue >= 1. */
grest_status grest_server_create(int64_t hbm_budget_bytes, int32_t lanes, int32_t max_queue,
                                 grest_server** out);

/* The same server whose lanes run batches: a free lane takes up to max_batch runnable
 * requests of distinct graphs (oldest first) and runs them as one grest_update_batch, each
 * graph on one of the lane's max_batch streams, so the one-workgroup stages of up to
 * max_batch updates go out as single launches.  Order, admission and results are as
 * above (a graph's result is the same alone or in any batch).  max_batch in [1,
 * GREST_BATCH_MAX], lanes * max_batch <= 256; max_batch = 1 is grest_server_create. */
grest_status grest_server_create_batched(int64_t hbm_budget_bytes, int32_t lanes, int32_t max_queue,
                                         int32_t max_batch, grest_server** out);

/* Attaches a state that already holds its pairs; *graph_id receives its id. */
grest_status grest_server_attach(grest_server* sv, grest_state* st, int32_t* graph_id);

/* Queues one update of graph `graph_id` (host arrays, copied before return; arguments as
 * for grest_update with where = GREST_HOST).  The change list's format is checked here
 * against the node count the graph will have once its queued requests have run
 * (EINVAL, nothing queued); checks that need the graph itself (an insertion of an
 * existing edge, a deletion of a missing one) surface in the request's completion
 * status, with that graph left unchanged.  `tag` is returned by grest_poll. */
grest_status grest_submit(grest_server* sv, int32_t graph_id, int64_t n_new, int64_t n_changes, const int32_t* ei,
                          const int32_t* ej, const int8_t* sign, const double* omega, uint64_t tag);

/* Copies up to `max` finished requests in completion order and removes them from the
 * server: tag, final status, submission and completion times.  Returns the count
 * (never blocks). */
int32_t grest_poll(grest_server* sv, int32_t max, uint64_t* tags, int32_t* status, int64_t* t_submit_ns,
                   int64_t* t_done_ns);

/* Detaches an idle graph (nothing of it queued or running; else GREST_EAGAIN): its
 * reservation is released, its state gets its original stream back and may be used
 * directly again; the id is not reused (submit to it: EINVAL). */
grest_status grest_server_detach(grest_server* sv, int32_t graph_id);

/* Device bytes reserved by the attached graphs (footprints plus the growth of queued
 * requests) and the budget; either pointer may be NULL. */
grest_status grest_server_memory(grest_server* sv, int64_t* reserved, int64_t* budget);

/* Blocks until every queued request has finished (they stay available to grest_poll). */
grest_status grest_server_drain(grest_server* sv);

/* Drains, stops the lanes, restores every attached state's stream.  The states stay
 * owned by the caller. */
void grest_server_destroy(grest_server* sv);

#ifdef __cplusplus
}
#endif

#endif /* GREST_H */
