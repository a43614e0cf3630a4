// Internal declarations shared by the HIP translation units of libgrest.
// Kernels are written for gfx950 (CDNA4): 64-wide wavefronts, 160 KB LDS per CU.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define GREST_WAVE 64

// Status bits raised by device code and surfaced through the deferred status word.
enum : int32_t {
  ST_BAD_FORMAT = 1 << 0,       // id out of range, i >= j, sign not +-1, delete on an appended node
  ST_DUPLICATE = 1 << 1,        // the same pair twice in one update
  ST_INSERT_EXISTING = 1 << 2,  // +1 on a pair that is already an edge
  ST_DELETE_MISSING = 1 << 3,   // -1 on a pair that is not an edge
  ST_NONFINITE = 1 << 4,        // NaN/Inf in the Gram matrix of an orthonormalisation
  ST_NOT_CONVERGED = 1 << 5,    // inverse iteration of the small eigensolver broke down
  ST_NONFINITE_H = 1 << 6,      // NaN/Inf in a matrix given to the small eigensolver
  ST_NUMERIC = ST_NONFINITE | ST_NOT_CONVERGED | ST_NONFINITE_H,
};

// ------------------------------------------------------------------------------------
// graph.hip: update of the stored graph (transition model of Sec. 2)
// ------------------------------------------------------------------------------------
void launch_fill_i64(int64_t* p, int64_t value, int64_t count, hipStream_t s);
void launch_fill_bytes0(void* p, size_t bytes, hipStream_t s);  // zero fill by a kernel
// exclusive scan of in[0..n) into out[0..n], out[n] = total; tmp >= scan_tmp_elems(n)
int64_t scan_tmp_elems(int64_t n);
void launch_scan_excl(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s);
// rows[0 .. pos[n_old + n_new]) = the appended rows and the old rows of Delta with an entry
// in an appended column, ascending (every row where Delta_2 Omega can be nonzero); flag
// and pos hold n_old + n_new + 1 entries, rows at most min(n_old + n_new, n_new + 2 nnz)
void launch_sketch_rows(int64_t n_old, int64_t n_new, const int64_t* dptr, const int32_t* dcol, int64_t* flag,
                        int64_t* pos, int64_t* scan_tmp, int32_t* rows, hipStream_t s);
// the same for the rows of Delta with any entry (where Delta_1 X can be nonzero); rows at
// most min(n_old + n_new, 2 nnz) entries
void launch_delta1_rows(int64_t n_old, int64_t n_new, const int64_t* dptr, const int32_t* dcol, int64_t* flag,
                        int64_t* pos, int64_t* scan_tmp, int32_t* rows, hipStream_t s);
// bits of a node id in the packed (row, column) keys of Delta
int delta_key_shift(int64_t n2);
// keys and signs of the two directed entries of every change (invalid: all-ones key and
// ST_BAD_FORMAT), and the per-row entry counts (cnt zeroed by the caller)
void launch_delta_keys(const int32_t* ei, const int32_t* ej, const int8_t* sg, int64_t nc, int64_t n_old,
                       int64_t n_new, int shift, uint64_t* keys, int8_t* vals, int64_t* cnt, int32_t* status,
                       hipStream_t s);
// longest row of Delta (changes at one node in one update) the grouping sorts; a longer
// row marks the update ST_BAD_FORMAT
constexpr int DELTA_LONG_MAX = 16384;
// The valid keys of kin (items entries; invalid ones are all ones) placed by row at the
// offsets dptr (cnt: the per-row counts, taken down to zero) into kout / vout with their
// signs, each row sorted by column.  list: n2 + 1 entries of scratch.
void launch_delta_group(const uint64_t* kin, const int8_t* vin, int64_t items, int shift, int64_t n2,
                        const int64_t* dptr, int64_t* cnt, uint64_t* kout, int8_t* vout, int64_t* list,
                        int32_t* status, hipStream_t s);
// column ids of the first *total sorted keys
void launch_delta_extract(const uint64_t* keys, int64_t items, const int64_t* total, int shift, int32_t* dcol,
                          hipStream_t s);
void launch_delta_rows(int64_t n_old, int64_t n_new, const int64_t* dptr, const int32_t* dcol, const int8_t* dsg,
                       int32_t* dins, const int64_t* rp_old, const int32_t* col_old, int64_t* newlen,
                       int32_t* status, hipStream_t s);
void launch_csr_merge(int64_t n_old, int64_t n_new, const int64_t* rp_old, const int32_t* col_old,
                      const int64_t* dptr, const int32_t* dcol, const int8_t* dsg, const int32_t* dins,
                      const int64_t* rp_new, int32_t* col_new, int64_t cap_m, hipStream_t s);
// degrees of the new graph, D^{-1/2} (0 for isolated nodes) and the maximum degree
void launch_degrees(int64_t n, const int64_t* rp, double* dinv_sqrt64, float* dinv_sqrt32,
                    int64_t* maxdeg, hipStream_t s);

// ------------------------------------------------------------------------------------
// spmm.hip: the product with the stored graph; delta.hip: products with the update
// ------------------------------------------------------------------------------------
enum OpKind : int32_t { OPK_ADJ = 0, OPK_LAP = 1, OPK_NLAP = 2 };

// Y[r, 0:w] = (op Z)[r, 0:w] for r in [0, n) with the L-form for Laplacians:
//   adj : sum_c Z[c]
//   lap : sum_c (Z[r] - Z[c])                 (= L Z)
//   nlap: s_r sum_c (s_r Z[r] - s_c Z[c])      (= L_n Z; isolated rows give Z[r])
// Z rows beyond nz_rows are treated as zero (padding).
// Rows with more than HEAVY_DEG entries (the hubs of power-law graphs) go to a kernel that
// splits each of them by entries over a whole workgroup; the others are row-split.
constexpr int64_t HEAVY_DEG = 128;
struct HeavyRows {
  const int32_t* rows;   // ids of the heavy rows, ascending
  const int64_t* count;  // their number (device)
  int64_t bound;         // an upper bound of the count known on the host (0: no heavy rows)
};
template <typename T>
void launch_spmm(int op, int64_t n, const int64_t* rp, const int32_t* col, const T* sc,
                 const T* Z, int64_t ldz, int64_t nz_rows, int w, T* Y, int64_t ldy, hipStream_t s,
                 const HeavyRows* heavy = nullptr);
// rows[0 .. *count) = the rows of the CSR with more than HEAVY_DEG entries, ascending; flag
// and pos hold n + 1 entries, scan_tmp scan_tmp_elems(n + 1)
void launch_heavy_rows(int64_t n, const int64_t* rp, int64_t* flag, int64_t* pos, int64_t* scan_tmp, int32_t* rows,
                       int64_t* count, hipStream_t s);

// Products with the update Delta of the tracked operator (rows grouped in dptr/dcol/dsg).
//   mode 0: V = Delta_1 Xbar            (only columns c < n_old, input X rows c)
//   mode 1: Y = Delta_2 Omega           (only columns c >= n_old, input rows c - n_old; only
//           the rows that can be nonzero are written, the others must be zero already)
//   mode 2: B = Delta_2^T M              (rows n_old.., all columns, input rows c)
//   mode 3: write Delta_2 densely into out[:, 0:S] (G-REST3)
// For lap/nlap the degree and scaling changes are included (see delta.hip).
// Mode 0 with acc_io: also acc_io[r] += V[r] on old rows with entries, acc_io[r] = V[r] on
// appended rows (turns a kept product of the old operator with X into the updated
// operator's product with the padded block).  Modes 0 and 1 with a row list (rows, *rcount
// <= bound on the device): only those rows are computed.  Mode 0: out must be zero elsewhere
// already, and acc_io's appended rows too; mode 1: the list must hold every row it writes.
// Modes 0 and 2 with heavy (the rows of Delta with more than HEAVY_DEG entries): those rows
// go to a workgroup each.
template <typename T>
void launch_delta_mul(int mode, int op, int64_t n_old, int64_t n_new, const int64_t* dptr,
                      const int32_t* dcol, const int8_t* dsg, const int64_t* maxdeg, const T* snew,
                      const T* in, int64_t ldin, int w, T* out, int64_t ldout, hipStream_t s,
                      T* acc_io = nullptr, int64_t ldacc = 0, const int32_t* rows = nullptr,
                      const int64_t* rcount = nullptr, int64_t bound = 0, const HeavyRows* heavy = nullptr);
// nlap: V = S'A'S' Xbar - [S A S X; 0] computed row by row from both graphs; with heavy
// (the new graph's heavy rows) those rows go to a workgroup each
template <typename T>
void launch_nlap_delta_x(int64_t n_old, int64_t n_new, const int64_t* rp_old, const int32_t* col_old,
                         const T* s_old, const int64_t* rp_new, const int32_t* col_new, const T* s_new,
                         const T* X, int64_t ldx, int k, T* V, int64_t ldv, hipStream_t s,
                         const HeavyRows* heavy = nullptr);

// ------------------------------------------------------------------------------------
// dense.hip: tall-skinny dense kernels (row-major blocks, n rows)
// ------------------------------------------------------------------------------------
// partial[g][a x b] = sum over the g-th row chunk of A[r, 0:a]^T B[r, 0:b]; then C = sum_g
// (fixed order).  ACC64 selects double accumulation inside a chunk.
int tn_num_chunks(int64_t n);
template <typename T, bool ACC64>
void launch_tn(int64_t n, const T* A, int64_t lda, int a, const T* B, int64_t ldb, int b,
               double* partial, double* C, hipStream_t s);
// Out[r, 0:b] = beta * Out[r, 0:b] + alpha * In[r, 0:a] @ M (M: a x b row-major, double)
// In and Out may alias when they are the same columns of the same rows (in-place, beta 0).
template <typename T>
void launch_apply(int64_t n, const T* In, int64_t ldin, int a, const double* M, int b, double alpha,
                  double beta, T* Out, int64_t ldout, hipStream_t s);
// mixed precision: BF16 MFMA with FP32 accumulation (FP32 inputs)
void launch_tn_bf16(int64_t n, const float* A, int64_t lda, int a, const float* B, int64_t ldb, int b,
                    double* partial, double* C, hipStream_t s);
template <typename T>
void launch_fill_rows(T* p, int64_t ld, int64_t row0, int64_t rows, int w, hipStream_t s);
// zero rows[0 .. *count) of a row-major block (bound: an upper bound of *count, sizes the grid)
template <typename T>
void launch_zero_listed_rows(T* p, int64_t ld, int w, const int32_t* rows, const int64_t* count, int64_t bound,
                             hipStream_t s);
// *dst = *src on the device
void launch_copy_i64(const int64_t* src, int64_t* dst, hipStream_t s);
// First CholQR round's apply fused with the second round's read pass (FP32 blocks):
// Out = W1 = [X | W] M1 (M1 (kx + w) x w; Out may be W), C = X^T W1 and G = W1^T W1 (FP64
// results).  kx, w multiples of 16 of the covered shapes, 16-byte aligned rows; false (and
// nothing queued) otherwise.  flag2 (optional) marks the rows where W can be nonzero.
bool apply_pip_ok(const float* X, int64_t ldx, int kx, const float* W, int64_t ldw, int w, const float* Out,
                  int64_t ldout);
bool launch_apply_pip(int64_t n, const float* X, int64_t ldx, int kx, const float* W, int64_t ldw, int w,
                      const int64_t* flag2, const double* M1, float* Out, int64_t ldout, double* partial, double* C,
                      double* G, hipStream_t s);
// Whether the fused FP32 CholQR2 against X of a block W in place (apply_pip_ok and a read
// pass launch_pip covers) reads W on the listed (flagged) rows alone in its first round:
// then W need not be zero elsewhere beforehand.
bool orth_reads_listed_rows_only(const float* X, int64_t ldx, int kx, const float* W, int64_t ldw, int w);
// H (d x d) += C diag(theta) C^T, C d x k row-major FP64; with md_old (the maximum degree of
// the old graph, device) also alpha (I - C C^T - Gn), alpha = 2 md_old, for the combinatorial
// Laplacian tracked in the L form (Gn d x d, may be null)
void launch_lowrank_h(int d, int k, const double* Cm, const double* theta, double* H, hipStream_t s,
                      const double* Gn = nullptr, const int64_t* md_old = nullptr);
// Zg[i] = Z[rows[i]], Dz[i] = (Delta Z)[rows[i]] for slots i < *count, zero rows up to bound
// (outputs bound x w, row-major, ld w); with lap, Dz[i] = (Delta_L Z)[rows[i]] instead, Delta_L
// = diag(degree changes) - Delta the change of the combinatorial Laplacian
template <typename T>
void launch_delta_gather(int64_t bound, const int32_t* rows, const int64_t* count, const int64_t* dptr,
                         const int32_t* dcol, const int8_t* dsg, const T* Z, int64_t ldz, int w, T* Zg, T* Dz,
                         hipStream_t s, bool lap = false);
// C (m x q) = A (m x p) B (p x q), row-major FP64
void launch_small_gemm(int m, int p, int q, const double* A, const double* B, double* C, hipStream_t s);
template <typename Tsrc, typename Tdst>
void launch_convert(const Tsrc* src, Tdst* dst, int64_t count, hipStream_t s);

// ------------------------------------------------------------------------------------
// small.hip: one-workgroup FP64 kernels on small matrices
// ------------------------------------------------------------------------------------
// Rank-revealing Cholesky of the Gram G (m x m) with diagonal pivoting.  Produces M
// (m x m) such that W M has orthonormal leading columns and zero trailing ones, and
// writes the kept count to *rank.  Columns are dropped when the pivot falls below
// (tol * scale)^2 where scale^2 = max(1, max_j (G_jj + colsq_j)); colsq may be null.
// With C (kc x m) the factored matrix is G - C^T C, the scale comes from diag(G), and the
// output Mout is the stacked (kc + m) x m matrix [-C M; M]; without C (kc = 0) Mout = M.
// The factor lives in registers and LDS (work is unused; pchol_work_elems is 0).
// m <= 128.
int64_t pchol_work_elems(int m, int kc);
void launch_pchol(int m, const double* G, const double* C, int kc, double tol, double* Mout, int32_t* rank,
                  int32_t* status, double* work, hipStream_t s);
// the same factor, without pivoting where that satisfies the truncation rule (pivoted
// otherwise); work holds a flag
void launch_pchol2(int m, const double* G, const double* C, int kc, double tol, double* Mout, int32_t* rank,
                  int32_t* status, double* work, hipStream_t s);
// one projection round in one pass: C = X^T W (working precision) and G = W^T W (FP64);
// returns false when the widths exceed what the kernel holds in registers.  With rows the
// pass covers rows[0 .. min(n, *nrows)) only (device count, n an upper bound), which is
// exact when W is zero on every other row.
template <typename T>
bool launch_pip(int64_t n, const T* X, int64_t ldx, int kx, const T* W, int64_t ldw, int w, double* partial,
                double* C, double* G, hipStream_t s, const int32_t* rows = nullptr,
                const int64_t* nrows = nullptr);
// Out = beta Out + alpha [In1 | In2] M  (In1: n x a1, In2: n x a2, a1 + a2 <= 128).  With
// flag2 the rows r with flag2[r] == 0 of In2 must be zero (they are then not read).  With
// rows (a device list, count in *nrows <= n) only the listed rows are computed.
template <typename T>
void launch_apply2(int64_t n, const T* In1, int64_t ld1, int a1, const T* In2, int64_t ld2, int a2,
                   const double* M, int b, double alpha, double beta, T* Out, int64_t ldout, hipStream_t s,
                   const int64_t* flag2 = nullptr, const int32_t* rows = nullptr, const int64_t* nrows = nullptr);
// Symmetric eigensolver of H (first base + rank[0] rows/cols used, ldh = d_full) and
// selection of kk pairs: which 0 = largest magnitude, 1 = smallest algebraic,
// 2 = largest algebraic.  Writes theta[kk] and F (d_full x kk, zero rows past the
// valid size); with drop_tol > 0 pairs whose value is at most drop_tol^2 max(1, max
// value) get theta 0 and a zero column, and *kept receives the number of the others.
// work: >= eig_work_elems(d_full) doubles.  Returns false (nothing launched) unless
// 1 <= d_full <= 128 and 1 <= kk <= 128.
// With rank2 the matrix is H restricted to the indices [0, base + *rank) followed by
// [seg2, seg2 + *rank2) (a basis of two packed blocks with dropped columns in between);
// F rows follow the same indices and the other rows are zero.
int64_t eig_work_elems(int d);
bool launch_small_eig(int d_full, int base, const int32_t* rank, const double* H, int which,
                      int kk, double drop_tol, double* theta, double* F, int32_t* kept,
                      double* work, int32_t* status, hipStream_t s, int seg2 = 0,
                      const int32_t* rank2 = nullptr);
// One graph's arguments of a CholQR factor (as launch_pchol2) or of a small eigensolve (as
// launch_small_eig), for the batched launches that serve many graphs at once.
struct CholJob {
  int m, kc;
  const double* G;
  const double* C;
  double tol;
  double* Mout;
  int32_t* rank;
  int32_t* status;
  double* work;
};
struct EigJob {
  int d_full, base, seg2, which, kk;
  const int32_t* rank;
  const int32_t* rank2;
  const double* H;
  double drop_tol;
  double* theta;
  double* F;
  int32_t* kept;
  double* work;
  int32_t* status;
  int b0_bisect, b0_vec;  // first block of the job in the batched grids (set by the prepare step)
};
bool small_eig_job_ok(const EigJob& j);  // the range launch_small_eig accepts
// Batched launches over nj jobs of different graphs: *_prepare orders the host array by
// kernel instance (and sets the block offsets); the caller copies it to dev (same layout,
// device memory) and calls *_launch with both on one stream.  Each job gets exactly the
// computation of its single-graph launch.
void chol_batch_prepare(CholJob* jobs, int nj);
void chol_batch_launch(const CholJob* jobs, const CholJob* dev, int nj, hipStream_t s);
void small_eig_batch_prepare(EigJob* jobs, int nj);
void small_eig_batch_launch(const EigJob* jobs, const EigJob* dev, int nj, hipStream_t s);
void batch_kernels_init();             // kernel attributes of the batched launches (idempotent)
int chol_job_key(const CholJob& j);    // kernel instances a job takes (the launch order key)
int eig_job_key(const EigJob& j);

// Many graphs' updates in lockstep (grest_update_batch): member threads meet at each
// one-workgroup stage and the last one to arrive launches that stage for all of them on
// the batch stream, which waits for the members' streams and which they wait for in turn.
struct BatchCtx;
BatchCtx* batch_create(int device, int max_members);
void batch_destroy(BatchCtx* bc);
void batch_begin(BatchCtx* bc, int members);
// called by a member at a stage; returns once that stage is queued for every member, with 0
// or the grest_status of a failed device call
int batch_chol(BatchCtx* bc, hipStream_t s, const CholJob& job);
int batch_small_eig(BatchCtx* bc, hipStream_t s, const EigJob& job);
void batch_leave(BatchCtx* bc);  // a member that has no stage left

// H = 0.5 (H + H^T) of a d x d matrix in place
void launch_symmetrize(int d, double* H, hipStream_t s);
template <typename T>
void launch_fill_random(T* p, int64_t ld, int64_t rows, int w, uint64_t seed, hipStream_t s);
// R[:, c] -= values[c] U[:, c] on an n x w block (the residual of tracked pairs)
template <typename T>
void launch_sub_scaled_cols(int64_t rows, int w, const double* values, const T* U, int64_t ldu, T* R, int64_t ldr,
                            hipStream_t s);
// Out = a P + b Q + c R on an n x w block (R may be null; Out may alias P, Q or R)
template <typename T>
void launch_lincomb3(int64_t rows, int w, double a, const T* P, int64_t ldp, double b, const T* Q, int64_t ldq,
                     double c, const T* R, int64_t ldr, T* Out, int64_t ldo, hipStream_t s);
// Y = a X + b Y on an n x w block
template <typename T>
void launch_axpby(int64_t rows, int w, double a, const T* X, int64_t ldx, double b, T* Y, int64_t ldy,
                  hipStream_t s);

// ------------------------------------------------------------------------------------
// noalloc.hip: the static workspace of the update that allocates nothing
// ------------------------------------------------------------------------------------
// largest change list of one grest_update_noalloc call, and the size of the device array
// that holds its change-list buffers (per device, for the life of the process)
constexpr int64_t kNoAllocMaxChanges = int64_t(1) << 18;
constexpr size_t kNoAllocScratchBytes = size_t(20) << 20;
// device address of that array on `device` (looked up once per device)
hipError_t noalloc_scratch(int device, void** out);

// ------------------------------------------------------------------------------------
// api.cpp: state accessors used by the server
// ------------------------------------------------------------------------------------
struct grest_state;
// capacities of a state's growing buffers and its current sizes
struct StateCaps {
  int64_t cap_n = 0, cap_m = 0, cap_nc = 0, cap_s = 0;
  int64_t n = 0, m = 0;
};
void state_caps(const grest_state* st, StateCaps* c);
// device bytes of the growing buffers at capacities c
int64_t state_bytes_for(const grest_state* st, const StateCaps& c);
// c advanced by one update of n_new nodes and nc changes that changes the stored entries
// by dm (the capacities grow as the update would grow them)
void state_caps_after(const grest_state* st, StateCaps* c, int64_t n_new, int64_t nc, int64_t dm);
// the caller's stream the state is bound to, or null when the state uses its own
void* state_user_stream(const grest_state* st);
// columns of the Gaussian test matrix an update needs (L + P for RSVD, else 0)
int64_t state_sketch_cols(const grest_state* st);
// Moves an idle state (nothing queued on its streams, e.g. right after grest_sync) onto
// another stream without waiting on the old one, which another state may be using.
// The state must not own its stream (attach has replaced an owned stream already).
void state_rebind_stream(grest_state* st, void* stream);
