// Host orchestration of the G-REST update behind the C interface of grest.h.
//
// One state owns, on one device: the graph as a double-buffered CSR, the dense
// basis buffers Z (two, row-major, ld = K + Dw) whose first K columns hold the
// tracked eigenvectors, the workspaces of the update, and the small FP64 matrices.
// An update is queued on the state's stream as: graph update and validation
// (one host wait for the status word), padding, Delta Xbar, the augmentation block
// (Delta_2 or the randomized basis R), two projections against Xbar, CholQR2 with
// FP64 Gram and pivoted Cholesky, (op Z), Z^T (op Z), the FP64 eigensolve, and the
// back-projection Z F into the other basis buffer.  The commit swaps buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/grest.h"
#include "grest_internal.h"

namespace {

thread_local char g_last_error[512] = "";

void set_err(const char* what, hipError_t e) {
  snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) {                            \
      set_err(#call, e_);                              \
      return e_ == hipErrorOutOfMemory ? GREST_ENOMEM : GREST_EDEVICE; \
    }                                                  \
  } while (0)

#define CHK(expr)                      \
  do {                                 \
    grest_status s_ = (expr);          \
    if (s_ != GREST_OK) return s_;     \
  } while (0)

constexpr int32_t VALIDATION_BITS = ST_BAD_FORMAT | ST_DUPLICATE | ST_INSERT_EXISTING | ST_DELETE_MISSING;

// Host-pinned results.  status, ranks and the Ritz values (which follow the struct in the
// same allocation, theta_pin) mirror the device block outbox, [status | ranks | pad | theta],
// so that the end of an update copies them back in one transfer.
struct Pinned {
  struct {
    int32_t vstatus;  // validation status of the update that used this slot
    int64_t m_new;
    int64_t hcount;   // heavy rows of the new graph
  } g[2];
  int32_t status;  // numerical status of the last update (copied at its end)
  int32_t ranks[8];
  int32_t pad;
};
constexpr size_t OUT_HDR = sizeof(int32_t) * 10;  // status, ranks, pad: theta starts here
static_assert(offsetof(Pinned, status) + OUT_HDR == sizeof(Pinned), "theta_pin follows Pinned::status at OUT_HDR");
static_assert(sizeof(Pinned) % sizeof(double) == 0, "theta_pin is 8-byte aligned");

template <typename P>
grest_status dalloc(P** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  HIPCHK(hipMalloc((void**)p, count * sizeof(P)));
  return GREST_OK;
}

template <typename P>
void dfree(P*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

}  // namespace

struct grest_state {
  grest_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  // set while the state's update is a member of a batch (grest_update_batch): its
  // one-workgroup stages are then launched with the other members'
  BatchCtx* batch = nullptr;
  int batch_err = 0;  // a failed device call of a batch round

  int prec = GREST_FP64;
  size_t es = 8;  // element size of the dense blocks
  int K = 0, op = 0, variant = 0, L = 0, Ls = 0, Dw = 0, D = 0, ldz = 0, ldy = 0;
  int ldq = 0;  // leading dimension of (op Z): D rounded up to 16 bytes, like ldz
  double tol = 1e-7;
  bool has_pairs = false;

  int64_t n = 0, m = 0;
  int64_t cap_n = 0, cap_m = 0, cap_nc = 0, cap_s = 0;

  int64_t* rp[2] = {nullptr, nullptr};
  int32_t* col[2] = {nullptr, nullptr};
  void* sc[2] = {nullptr, nullptr};  // D^{-1/2} per node, working precision
  int gcur = 0;

  void* z[2] = {nullptr, nullptr};
  int zcur = 0;
  void* aux = nullptr;   // (op Z), cap_n x D with leading dimension ldq
  void* ybuf = nullptr;  // sketch Y = Delta_2 Omega, cap_n x ldy, zero outside the listed rows
  void* mbuf = nullptr;  // its orthonormal basis M, cap_n x ldy
  bool y_clean = false;  // ybuf is zero outside srows[0 .. *srows_cnt)
  int64_t* srows_cnt = nullptr;  // device count of the last sketch row list
  int64_t srows_bound = 0;       // host upper bound of that count
  void* bt = nullptr;    // Delta_2^T M, cap_s x Ls
  void* omega_t = nullptr;
  double* omega64 = nullptr;

  // Graph stage of an update (change list sorted into Delta, validation, merge into the
  // other CSR buffer).  It runs on gstream, which is the state's stream unless the
  // overlap mode gives it a stream of its own, so that it runs while the device finishes
  // the previous update.  What the rest of the update reads (Delta's CSR, the status word
  // of the validation) comes in two slots used by alternate updates; the arrays only
  // the graph stage touches are single.
  hipStream_t gstream = nullptr;
  bool overlap = false;
  int dslot = 0;               // slot of the update in progress
  bool prev_rejected = false;  // the last update call failed its validation
  hipEvent_t gev[2] = {};      // graph stage of the slot's update done (results on the host)
  hipEvent_t endev[2] = {};    // every kernel of the slot's update done
  hipEvent_t gate[2] = {};     // the slot's update has reached its small eigensolve
  hipEvent_t ogate[2] = {};    // the slot's update has read its old graph for the last time
  bool ogate_recorded[2] = {false, false};
  bool end_recorded[2] = {false, false}, gate_recorded[2] = {false, false};
  int32_t *d_ei = nullptr, *d_ej = nullptr;
  int8_t* d_sg = nullptr;
  int64_t *dcnt = nullptr, *newlen = nullptr, *scan_tmp = nullptr;
  int64_t* dptr[2] = {nullptr, nullptr};
  int32_t* dcol[2] = {nullptr, nullptr};
  int8_t* dsg[2] = {nullptr, nullptr};
  int32_t* vstat[2] = {nullptr, nullptr};  // validation bits per slot
  uint64_t *dkey_in = nullptr, *dkey_out = nullptr;  // packed (row, column) keys of Delta
  int32_t* dins = nullptr;
  int8_t* dsg_tmp = nullptr;
  // row lists of the sparse projection rounds (flags, positions, scan workspace): the
  // sketch's (r*) and Delta_1 X's (d*)
  int64_t *rflag = nullptr, *rpos = nullptr, *rscan_tmp = nullptr;
  int64_t *dflag = nullptr, *dpos = nullptr, *dscan_tmp = nullptr;
  int32_t* srows = nullptr;  // rows where the sketch Delta_2 Omega can be nonzero
  int32_t* drows = nullptr;  // rows where Delta_1 X can be nonzero

  double *C1 = nullptr, *C2 = nullptr, *Gm = nullptr, *Mchol = nullptr, *H = nullptr, *F = nullptr;
  double* Msk = nullptr;  // coefficients of R = [Xbar Y1] (Mchol U_L), (K + Ls) x L
  double* M1buf = nullptr;  // first-round factor of a fused CholQR2 (same shape as Mchol)
  // low-rank projection: the listed rows of Z and of Delta Z (2 cap_nc x D each), and
  // C = Z^T Xbar (D x K)
  int proj = GREST_PROJ_EXACT;
  void* zg = nullptr;
  void* dz = nullptr;
  double* Clr = nullptr;
  double *Fb = nullptr, *thetab = nullptr, *partial = nullptr, *eigwork = nullptr;
  // outbox: status word, kept column counts and Ritz values in one device block (the
  // layout of Pinned from status on), carved into status, ranks and theta
  void* outbox = nullptr;
  double* theta = nullptr;
  int32_t* ranks = nullptr;
  int32_t* status = nullptr;
  int64_t* maxdeg[2] = {nullptr, nullptr};  // largest degree of CSR buffer b
  // rows of CSR buffer b with more than HEAVY_DEG entries (multiplied by a workgroup each),
  // their count on the device and on the host; flag, position and scan workspaces
  int32_t* hrows[2] = {nullptr, nullptr};
  int64_t* hcnt[2] = {nullptr, nullptr};
  int64_t hcnt_host[2] = {0, 0};
  int64_t *hflag = nullptr, *hpos = nullptr, *hscan = nullptr;
  // rows of the current Delta with more than HEAVY_DEG entries (count on the device)
  int32_t* dhrows = nullptr;
  int64_t* dhcnt = nullptr;
  Pinned* pin = nullptr;
  double* theta_pin = nullptr;
  int32_t deferred = 0;
  int64_t partial_elems = 0;
  // adjacency only: aux[:, 0:K] holds A X for the current graph and tracked block (kept
  // from the last back-projection), so the next update multiplies only the new columns
  bool ax_valid = false;
  // low-rank states only: the stored graph has been released (grest_release_graph); updates
  // keep Delta alone, and the checks that need the old graph are not made
  bool graph_free = false;
  // restart policy (grest_set_restart): every rs_every updates the drift of the pairs is
  // measured; past a threshold, and at least rs_gap updates after the last (re)start,
  // the pairs are recomputed from scratch by the initial eigensolver
  double rs_tol_resid = 0.0, rs_tol_orth = 0.0;
  int rs_every = 0, rs_gap = 0, rs_iters = 0;
  uint64_t rs_seed = 0;
  int64_t rs_since_check = 0, rs_since_start = 0, rs_count = 0;
  double rs_last_orth = -1.0, rs_last_resid = -1.0;
  int32_t ax_age = 0;  // updates since the last full-width product
  // the last run of the initial eigensolver: products with the operator, final residual
  int32_t last_init_products = 0;
  double last_init_resid = -1.0;

  // optional stage timing with HIP events on the state's stream; two sets of events, used
  // by alternate updates, so that an update's events are read (at the next update's
  // validation wait, when they have completed) before they are recorded again
  static constexpr int NSTAGE = 8;
  bool prof = false;
  int pslot = 0;
  bool prof_pending[2] = {false, false};
  hipEvent_t pev[2][NSTAGE + 1] = {};
  hipEvent_t gend[2] = {};    // end of the graph stage (on gstream)
  hipEvent_t kev[2][2] = {};  // around the (op Z) product alone
  double stage_ms[NSTAGE] = {};
  double spmm_ms = 0.0;
  int64_t spmm_cols[2] = {0, 0};  // width of the (op Z) product per event set
  int64_t prof_spmm_cols = 0;
  int64_t prof_updates = 0;
  bool marking = false;
  bool stage_marks = true;  // false: only the events around the sparse product
};

namespace {

void mark(grest_state* st, int i) {
  if (st->marking && st->stage_marks)
    (void)hipEventRecord(st->pev[st->pslot][i], i == 0 ? st->gstream : st->stream);
}

void mark_spmm(grest_state* st, int i) {
  if (st->marking) (void)hipEventRecord(st->kev[st->pslot][i], st->stream);
}

// add the stage times of the update that used event set `slot` (its events have completed)
void prof_collect_slot(grest_state* st, int slot) {
  if (!st->prof_pending[slot]) return;
  for (int i = 0; i < grest_state::NSTAGE && st->stage_marks; ++i) {
    float ms = 0.f;
    hipEvent_t e1 = i == 0 ? st->gend[slot] : st->pev[slot][i + 1];
    if (hipEventElapsedTime(&ms, st->pev[slot][i], e1) == hipSuccess) st->stage_ms[i] += ms;
  }
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, st->kev[slot][0], st->kev[slot][1]) == hipSuccess) st->spmm_ms += ms;
  st->prof_spmm_cols += st->spmm_cols[slot];
  st->prof_updates += 1;
  st->prof_pending[slot] = false;
}

// after a full wait on the stream
void prof_collect(grest_state* st) {
  prof_collect_slot(st, st->pslot ^ 1);
  prof_collect_slot(st, st->pslot);
}

}  // namespace

namespace {

int64_t round_up(int64_t v, int64_t q) { return ((v + q - 1) / q) * q; }

// wait for everything queued on the state's streams
grest_status sync_all(grest_state* st) {
  HIPCHK(hipStreamSynchronize(st->stream));
  if (st->gstream && st->gstream != st->stream) HIPCHK(hipStreamSynchronize(st->gstream));
  return GREST_OK;
}

grest_status alloc_node_arrays(grest_state* st, int64_t cap_n) {
  const size_t es = st->es;
  for (int b = 0; b < 2; ++b) {
    CHK(dalloc(&st->rp[b], cap_n + 1));
    CHK(dalloc((char**)&st->sc[b], cap_n * es));
    CHK(dalloc((char**)&st->z[b], (size_t)cap_n * st->ldz * es));
  }
  if (!st->graph_free) CHK(dalloc((char**)&st->aux, (size_t)cap_n * st->ldq * es));
  if (st->variant == GREST_RSVD) {
    CHK(dalloc((char**)&st->ybuf, (size_t)cap_n * st->ldy * es));
    CHK(dalloc((char**)&st->mbuf, (size_t)cap_n * st->ldy * es));
  }
  st->y_clean = false;
  CHK(dalloc(&st->dcnt, cap_n + 1));
  CHK(dalloc(&st->dptr[0], cap_n + 1));
  CHK(dalloc(&st->dptr[1], cap_n + 1));
  CHK(dalloc(&st->newlen, cap_n + 1));
  CHK(dalloc(&st->scan_tmp, scan_tmp_elems(cap_n + 1) + 16));
  CHK(dalloc(&st->rflag, cap_n + 1));
  CHK(dalloc(&st->rpos, cap_n + 1));
  CHK(dalloc(&st->rscan_tmp, scan_tmp_elems(cap_n + 1) + 16));
  CHK(dalloc(&st->dflag, cap_n + 1));
  CHK(dalloc(&st->dpos, cap_n + 1));
  CHK(dalloc(&st->dscan_tmp, scan_tmp_elems(cap_n + 1) + 16));
  CHK(dalloc(&st->srows, cap_n + 1));
  CHK(dalloc(&st->drows, cap_n + 1));
  for (int b = 0; b < 2; ++b) CHK(dalloc(&st->hrows[b], cap_n + 1));
  CHK(dalloc(&st->dhrows, cap_n + 1));
  CHK(dalloc(&st->hflag, cap_n + 1));
  CHK(dalloc(&st->hpos, cap_n + 1));
  CHK(dalloc(&st->hscan, scan_tmp_elems(cap_n + 1) + 16));
  st->cap_n = cap_n;
  return GREST_OK;
}

grest_status alloc_edge_arrays(grest_state* st, int64_t cap_m) {
  for (int b = 0; b < 2; ++b) {
    CHK(dalloc(&st->col[b], cap_m));
    HIPCHK(hipMemsetAsync(st->col[b], 0, (size_t)cap_m * sizeof(int32_t), st->stream));
  }
  st->cap_m = cap_m;
  return GREST_OK;
}

// The low-rank form's gathered rows of Z and Delta Z: one per row of Delta with an entry,
// at most min(n', 2 x changes) <= min(node capacity, 2 x change capacity); reallocated
// when either capacity grows (both callers have synchronised the state)
grest_status alloc_gather_arrays(grest_state* st) {
  dfree(st->zg);
  dfree(st->dz);
  if (st->proj != GREST_PROJ_LOWRANK) return GREST_OK;
  const int64_t rows = std::max<int64_t>(1, std::min<int64_t>(2 * st->cap_nc, st->cap_n));
  CHK(dalloc((char**)&st->zg, (size_t)rows * st->D * st->es));
  CHK(dalloc((char**)&st->dz, (size_t)rows * st->D * st->es));
  return GREST_OK;
}

grest_status alloc_change_arrays(grest_state* st, int64_t cap_nc) {
  CHK(sync_all(st));  // queued work may still read the old arrays
  dfree(st->d_ei); dfree(st->d_ej); dfree(st->d_sg);
  dfree(st->dkey_in); dfree(st->dkey_out);
  dfree(st->dcol[0]); dfree(st->dcol[1]); dfree(st->dins); dfree(st->dsg_tmp); dfree(st->dsg[0]); dfree(st->dsg[1]);
  CHK(dalloc(&st->d_ei, cap_nc));
  CHK(dalloc(&st->d_ej, cap_nc));
  CHK(dalloc(&st->d_sg, cap_nc));
  CHK(dalloc(&st->dkey_in, 2 * cap_nc));
  CHK(dalloc(&st->dkey_out, 2 * cap_nc));
  for (int b = 0; b < 2; ++b) {
    CHK(dalloc(&st->dcol[b], 2 * cap_nc));
    CHK(dalloc(&st->dsg[b], 2 * cap_nc));
  }
  CHK(dalloc(&st->dins, 2 * cap_nc));
  CHK(dalloc(&st->dsg_tmp, 2 * cap_nc));
  st->cap_nc = cap_nc;
  return alloc_gather_arrays(st);
}

grest_status alloc_sketch_arrays(grest_state* st, int64_t cap_s) {
  CHK(sync_all(st));  // queued work may still read the old arrays
  dfree(st->bt); dfree(st->omega_t); dfree(st->omega64);
  if (st->variant != GREST_RSVD) { st->cap_s = cap_s; return GREST_OK; }
  CHK(dalloc((char**)&st->bt, (size_t)cap_s * st->Ls * st->es));
  CHK(dalloc((char**)&st->omega_t, (size_t)cap_s * st->Ls * st->es));
  CHK(dalloc(&st->omega64, (size_t)cap_s * st->Ls));
  st->cap_s = cap_s;
  return GREST_OK;
}

// device bytes of every buffer of the state (the same list free_all releases)
int64_t device_bytes(const grest_state* st) {
  int64_t total = 0;
  auto add = [&](const void* p) {
    size_t sz = 0;
    if (p && hipMemPtrGetInfo(const_cast<void*>(p), &sz) == hipSuccess) total += (int64_t)sz;
  };
  for (int b = 0; b < 2; ++b) { add(st->rp[b]); add(st->col[b]); add(st->sc[b]); add(st->z[b]); }
  add(st->aux); add(st->ybuf); add(st->mbuf); add(st->srows_cnt); add(st->bt); add(st->omega_t); add(st->omega64);
  add(st->d_ei); add(st->d_ej); add(st->d_sg);
  add(st->dcnt); add(st->newlen); add(st->scan_tmp); add(st->srows); add(st->drows);
  add(st->rflag); add(st->rpos); add(st->rscan_tmp); add(st->dflag); add(st->dpos); add(st->dscan_tmp);
  add(st->hrows[0]); add(st->hrows[1]); add(st->hcnt[0]); add(st->hcnt[1]); add(st->hflag); add(st->hpos);
  add(st->dhrows); add(st->dhcnt);
  add(st->hscan);
  add(st->dkey_in); add(st->dkey_out); add(st->dins); add(st->dsg_tmp);
  for (int b = 0; b < 2; ++b) {
    add(st->dptr[b]); add(st->dcol[b]); add(st->dsg[b]); add(st->vstat[b]); add(st->maxdeg[b]);
  }
  add(st->C1); add(st->C2); add(st->Gm); add(st->Mchol); add(st->H); add(st->F); add(st->Msk); add(st->M1buf);
  add(st->zg); add(st->dz); add(st->Clr);
  add(st->outbox); add(st->Fb); add(st->thetab); add(st->partial); add(st->eigwork);
  return total;
}

void free_all(grest_state* st) {
  for (int b = 0; b < 2; ++b) {
    dfree(st->rp[b]); dfree(st->col[b]); dfree(st->sc[b]); dfree(st->z[b]);
  }
  dfree(st->aux); dfree(st->ybuf); dfree(st->mbuf); dfree(st->srows_cnt); dfree(st->bt); dfree(st->omega_t); dfree(st->omega64);
  dfree(st->d_ei); dfree(st->d_ej); dfree(st->d_sg);
  dfree(st->dcnt); dfree(st->newlen); dfree(st->scan_tmp); dfree(st->srows); dfree(st->drows);
  dfree(st->rflag); dfree(st->rpos); dfree(st->rscan_tmp); dfree(st->dflag); dfree(st->dpos); dfree(st->dscan_tmp);
  dfree(st->hrows[0]); dfree(st->hrows[1]); dfree(st->hcnt[0]); dfree(st->hcnt[1]); dfree(st->hflag);
  dfree(st->dhrows); dfree(st->dhcnt);
  dfree(st->hpos); dfree(st->hscan);
  dfree(st->dkey_in); dfree(st->dkey_out); dfree(st->dins); dfree(st->dsg_tmp);
  for (int b = 0; b < 2; ++b) {
    dfree(st->dptr[b]); dfree(st->dcol[b]); dfree(st->dsg[b]); dfree(st->vstat[b]); dfree(st->maxdeg[b]);
    if (st->gev[b]) (void)hipEventDestroy(st->gev[b]);
    if (st->endev[b]) (void)hipEventDestroy(st->endev[b]);
    if (st->gate[b]) (void)hipEventDestroy(st->gate[b]);
    if (st->ogate[b]) (void)hipEventDestroy(st->ogate[b]);
    st->gev[b] = st->endev[b] = st->gate[b] = st->ogate[b] = nullptr;
  }
  dfree(st->C1); dfree(st->C2); dfree(st->Gm); dfree(st->Mchol); dfree(st->H); dfree(st->F); dfree(st->Msk); dfree(st->M1buf);
  dfree(st->zg); dfree(st->dz); dfree(st->Clr);
  dfree(st->outbox); dfree(st->Fb); dfree(st->thetab); dfree(st->partial); dfree(st->eigwork);
  st->theta = nullptr;
  st->ranks = nullptr;
  st->status = nullptr;
  if (st->pin) (void)hipHostFree(st->pin);  // theta_pin lives in the same allocation
  st->pin = nullptr;
  st->theta_pin = nullptr;
}

// the heavy rows of CSR buffer b (its graph in place), with their count copied to the host
grest_status heavy_rows_sync(grest_state* st, int b) {
  if (st->graph_free) {
    st->hcnt_host[b] = 0;
    return GREST_OK;
  }
  launch_heavy_rows(st->n, st->rp[b], st->hflag, st->hpos, st->hscan, st->hrows[b], st->hcnt[b], st->stream);
  HIPCHK(hipMemcpyAsync(&st->hcnt_host[b], st->hcnt[b], sizeof(int64_t), hipMemcpyDeviceToHost, st->stream));
  HIPCHK(hipStreamSynchronize(st->stream));
  return GREST_OK;
}

HeavyRows heavy_of(const grest_state* st, int b) { return HeavyRows{st->hrows[b], st->hcnt[b], st->hcnt_host[b]}; }

// Grow node-indexed buffers, keeping the current graph and basis.
grest_status grow_nodes(grest_state* st, int64_t need) {
  int64_t cap = std::max<int64_t>(need, st->cap_n + st->cap_n / 2);
  if (cap >= INT32_MAX) cap = INT32_MAX - 1;  // node ids are int32
  if (cap < need) return GREST_EINVAL;
  CHK(sync_all(st));
  st->ax_valid = false;  // the product buffer is reallocated below
  int64_t* rp_old = st->rp[st->gcur];
  void* z_old = st->z[st->zcur];
  void* sc_old = st->sc[st->gcur];
  int64_t* rp_keep[2] = {st->rp[0], st->rp[1]};
  void* z_keep[2] = {st->z[0], st->z[1]};
  void* sc_keep[2] = {st->sc[0], st->sc[1]};
  st->rp[0] = st->rp[1] = nullptr;
  st->z[0] = st->z[1] = nullptr;
  st->sc[0] = st->sc[1] = nullptr;
  dfree(st->aux); dfree(st->ybuf); dfree(st->mbuf); dfree(st->dcnt); dfree(st->dptr[0]); dfree(st->dptr[1]);
  dfree(st->newlen); dfree(st->scan_tmp); dfree(st->rflag); dfree(st->rpos); dfree(st->rscan_tmp);
  dfree(st->dflag); dfree(st->dpos); dfree(st->dscan_tmp);
  dfree(st->srows); dfree(st->drows);
  dfree(st->hrows[0]); dfree(st->hrows[1]); dfree(st->hflag); dfree(st->hpos); dfree(st->hscan);
  dfree(st->dhrows);
  CHK(alloc_node_arrays(st, cap));
  CHK(alloc_gather_arrays(st));
  HIPCHK(hipMemcpyAsync(st->rp[st->gcur], rp_old, (st->n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice,
                        st->stream));
  HIPCHK(hipMemcpyAsync(st->sc[st->gcur], sc_old, st->n * st->es, hipMemcpyDeviceToDevice, st->stream));
  HIPCHK(hipMemcpyAsync(st->z[st->zcur], z_old, (size_t)st->n * st->ldz * st->es, hipMemcpyDeviceToDevice,
                        st->stream));
  CHK(heavy_rows_sync(st, st->gcur));
  HIPCHK(hipStreamSynchronize(st->stream));
  for (int b = 0; b < 2; ++b) { dfree(rp_keep[b]); dfree(z_keep[b]); dfree(sc_keep[b]); }
  return GREST_OK;
}

grest_status grow_edges(grest_state* st, int64_t need) {
  int64_t cap = std::max<int64_t>(need, st->cap_m + st->cap_m / 2);
  CHK(sync_all(st));
  int32_t* keep[2] = {st->col[0], st->col[1]};
  st->col[0] = st->col[1] = nullptr;
  CHK(alloc_edge_arrays(st, cap));
  HIPCHK(hipMemcpyAsync(st->col[st->gcur], keep[st->gcur], st->m * sizeof(int32_t), hipMemcpyDeviceToDevice,
                        st->stream));
  HIPCHK(hipStreamSynchronize(st->stream));
  dfree(keep[0]);
  dfree(keep[1]);
  return GREST_OK;
}

// ---------------------------------------------------------------------------------
// the update, templated on the element type of the dense blocks
// ---------------------------------------------------------------------------------
template <typename T>
struct Blocks {
  T* Zc;  // current basis buffer (X in columns 0..K)
  T* Zn;  // next basis buffer
  T* W;   // columns K .. K+Dw of Zc
  T* Y;   // sketch buffer
  T* aux;
};

template <typename T>
Blocks<T> blocks(grest_state* st) {
  Blocks<T> b;
  b.Zc = (T*)st->z[st->zcur];
  b.Zn = (T*)st->z[st->zcur ^ 1];
  b.W = b.Zc + st->K;
  b.Y = (T*)st->ybuf;
  b.aux = (T*)st->aux;
  return b;
}

// The one-workgroup stages of an update: launched on the state's stream, or, while the
// update is a member of a batch, handed to the batch, which launches them with the other
// members' (the same kernels with the same arguments).
void pchol2_stage(grest_state* st, int m, const double* G, const double* C, int kc, double* Mout, int32_t* rank) {
  if (!st->batch) {
    launch_pchol2(m, G, C, kc, st->tol, Mout, rank, st->status, st->eigwork, st->stream);
    return;
  }
  const CholJob j{m, kc, G, C, st->tol, Mout, rank, st->status, st->eigwork};
  if (int rc = batch_chol(st->batch, st->stream, j)) st->batch_err = rc;
}

bool small_eig_stage(grest_state* st, int d_full, int base, const int32_t* rank, const double* H, int which, int kk,
                     double drop_tol, double* theta, double* F, int32_t* kept, int seg2 = 0,
                     const int32_t* rank2 = nullptr) {
  if (!st->batch)
    return launch_small_eig(d_full, base, rank, H, which, kk, drop_tol, theta, F, kept, st->eigwork, st->status,
                            st->stream, seg2, rank2);
  EigJob j{};
  j.d_full = d_full; j.base = base; j.seg2 = seg2; j.which = which; j.kk = kk;
  j.rank = rank; j.rank2 = rank2; j.H = H; j.drop_tol = drop_tol;
  j.theta = theta; j.F = F; j.kept = kept; j.work = st->eigwork; j.status = st->status;
  if (!small_eig_job_ok(j)) return false;
  if (int rc = batch_small_eig(st->batch, st->stream, j)) st->batch_err = rc;
  return true;
}

// Orthonormal basis of (I - Xbar Xbar^T) W in place (W: n x w, ld), two rounds of block
// Gram-Schmidt with the Pythagorean Gram (CholQR2 against Xbar): each round reads
// [Xbar W] once for C = Xbar^T W and the FP64 Gram G = W^T W, factors G - C^T C by
// rank-revealing pivoted Cholesky in FP64, and writes W <- (W - Xbar C) M in one pass.
// The kept column counts of the two rounds go to ranks[slot] and ranks[slot + 1].
// With rows (a device list of at most rows_bound rows, count in *nrows) W is zero outside
// those rows, and the first round's read pass covers them only.
// With Wout the first round reads W and writes Wout (same leading dimension), and the
// second round works on Wout in place; flag2 (with rows) marks the rows of W that can be
// nonzero, so the first round's apply does not read the others.
// Without last_apply the second round stops at its factor: the basis is then
// [X Wout] Mchol, which the caller applies itself.
// FP32 blocks of the covered shapes fuse the first round's apply with the second round's
// read pass (launch_apply_pip): W1 is written and its Gram products are formed from the
// registers that hold it, which saves reading it back.
template <typename T>
void orth_against(grest_state* st, int64_t n, const T* X, int64_t ldx, int kx, T* W, int64_t ldw, int w, int slot,
                  const int32_t* rows = nullptr, const int64_t* nrows = nullptr, int64_t rows_bound = 0,
                  T* Wout = nullptr, const int64_t* flag2 = nullptr, bool last_apply = true) {
  hipStream_t s = st->stream;
  if constexpr (sizeof(T) == 4) {
    T* Wo = Wout ? Wout : W;
    if (apply_pip_ok(X, ldx, kx, W, ldw, w, Wo, ldw)) {
      if (!(rows ? launch_pip<T>(rows_bound, X, ldx, kx, W, ldw, w, st->partial, st->C1, st->Gm, s, rows, nrows)
                 : launch_pip<T>(n, X, ldx, kx, W, ldw, w, st->partial, st->C1, st->Gm, s))) {
        launch_tn<T, false>(n, X, ldx, kx, W, ldw, w, st->partial, st->C1, s);
        launch_tn<T, true>(n, W, ldw, w, W, ldw, w, st->partial, st->Gm, s);
      }
      pchol2_stage(st, w, st->Gm, st->C1, kx, st->M1buf, st->ranks + slot);
      launch_apply_pip(n, X, ldx, kx, W, ldw, w, flag2, st->M1buf, Wo, ldw, st->partial, st->C1, st->Gm, s);
      pchol2_stage(st, w, st->Gm, st->C1, kx, st->Mchol, st->ranks + slot + 1);
      if (last_apply) launch_apply2<T>(n, X, ldx, kx, Wo, ldw, w, st->Mchol, w, 1.0, 0.0, Wo, ldw, s);
      return;
    }
  }
  for (int round = 0; round < 2; ++round) {
    const bool sparse = round == 0 && rows;
    T* Win = (round == 1 && Wout) ? Wout : W;
    T* Wo = Wout ? Wout : W;
    if (!(sparse ? launch_pip<T>(rows_bound, X, ldx, kx, Win, ldw, w, st->partial, st->C1, st->Gm, s, rows, nrows)
                 : launch_pip<T>(n, X, ldx, kx, Win, ldw, w, st->partial, st->C1, st->Gm, s))) {
      if (st->prec == GREST_FP64) launch_tn<T, true>(n, X, ldx, kx, Win, ldw, w, st->partial, st->C1, s);
      else launch_tn<T, false>(n, X, ldx, kx, Win, ldw, w, st->partial, st->C1, s);
      launch_tn<T, true>(n, Win, ldw, w, Win, ldw, w, st->partial, st->Gm, s);
    }
    pchol2_stage(st, w, st->Gm, st->C1, kx, st->Mchol, st->ranks + slot + round);
    if (round == 1 && !last_apply) break;
    if (round == 0 && rows && Wout) {
      // W is zero off the listed rows and goes to another buffer: Wout = X (-C M) over
      // every row, then Wout += W M on the listed rows alone
      launch_apply2<T>(n, X, ldx, kx, X, ldx, 0, st->Mchol, w, 1.0, 0.0, Wo, ldw, s);
      launch_apply2<T>(rows_bound, W, ldw, w, W, ldw, 0, st->Mchol + (size_t)kx * w, w, 1.0, 1.0, Wo, ldw, s,
                       nullptr, rows, nrows);
    } else {
      launch_apply2<T>(n, X, ldx, kx, Win, ldw, w, st->Mchol, w, 1.0, 0.0, Wo, ldw, s,
                       round == 0 ? flag2 : nullptr);
    }
  }
}

// rank-revealing CholQR2 of W (n x w, ld) in place, without a block to project against
template <typename T>
void cholqr2(grest_state* st, int64_t n, T* W, int64_t ldw, int w, int slot) {
  for (int round = 0; round < 2; ++round) {
    launch_tn<T, true>(n, W, ldw, w, W, ldw, w, st->partial, st->Gm, st->stream);
    launch_pchol(w, st->Gm, nullptr, 0, st->tol, st->Mchol, st->ranks + slot + round, st->status, st->eigwork,
                 st->stream);
    launch_apply<T>(n, W, ldw, w, st->Mchol, w, 1.0, 0.0, W, ldw, st->stream);
  }
}

// With reuse, aux[:, 0:K] already holds (op) Xbar for the updated operator (the kept
// product of the old operator with X plus Delta_1 X, added during the Delta Xbar stage),
// and only the other columns of Z go through the sparse product.
// The basis may hold two packed blocks with dropped columns between them: the small
// eigensolve then works on the kept columns [0, base + *rank_slot) and
// [seg2, seg2 + *rank2).
struct LowRankIn {  // Delta's CSR and the list of its nonempty rows (count on the device)
  const int64_t* dptr;
  const int32_t* dcol;
  const int8_t* dsg;
  const int32_t* rows;
  const int64_t* count;
  int64_t bound;
};

template <typename T>
grest_status rayleigh_ritz(grest_state* st, int64_t n2, const int64_t* rp, const int32_t* col, const T* sc,
                           int base, int32_t* rank_slot, bool reuse, int seg2 = 0, const int32_t* rank2 = nullptr,
                           int gate_slot = -1, const LowRankIn* lr = nullptr) {
  Blocks<T> b = blocks<T>(st);
  if (lr) {
    // low-rank projected matrix (eq. RR_eigen_graph_upd_main3): H = C Theta C^T + Z^T Delta Z
    // with C = Z^T Xbar and the previous Ritz values Theta; Delta Z is nonzero only on the
    // rows of Delta with an entry, so Z^T Delta Z is a product over those rows, gathered
    T* Zg = (T*)st->zg;
    T* Dz = (T*)st->dz;
    mark_spmm(st, 0);  // no sparse product with the whole graph
    mark_spmm(st, 1);
    st->spmm_cols[st->pslot] = 0;
    mark(st, 5);
    // the products take the precision of the exact form's H: split BF16 in the mixed mode,
    // FP32 MFMA for FP32 blocks, FP64 MFMA for FP64 blocks
    auto product = [&](int64_t rows, const T* A, int64_t lda, int a, const T* B, int64_t ldb, int bw, double* out) {
      if constexpr (sizeof(T) == 4) {
        if (st->prec == GREST_MIXED)
          launch_tn_bf16(rows, A, lda, a, B, ldb, bw, st->partial, out, st->stream);
        else
          launch_tn<T, false>(rows, A, lda, a, B, ldb, bw, st->partial, out, st->stream);
      } else {
        launch_tn<T, true>(rows, A, lda, a, B, ldb, bw, st->partial, out, st->stream);
      }
    };
    const bool lap = st->op == GREST_OP_LAP;
    // the Laplacian's form below multiplies I - C C^T - Z_new^T Z_new by the shift alpha =
    // 2 d_max, which would scale the error of a split-BF16 product up to alpha times itself:
    // there C and the Gram of the appended rows take FP64 accumulation
    if (lap)
      launch_tn<T, true>(n2, b.Zc, st->ldz, st->D, b.Zc, st->ldz, st->K, st->partial, st->Clr, st->stream);
    else
      product(n2, b.Zc, st->ldz, st->D, b.Zc, st->ldz, st->K, st->Clr);
    launch_delta_gather<T>(lr->bound, lr->rows, lr->count, lr->dptr, lr->dcol, lr->dsg, b.Zc, st->ldz, st->D, Zg,
                           Dz, st->stream, lap);
    if (lr->bound > 0) {
      product(lr->bound, Zg, st->D, st->D, Dz, st->D, st->D, st->H);
    } else {
      launch_fill_rows<double>(st->H, st->D, 0, st->D, st->D, st->stream);
    }
    if (lap) {
      // The truncated form approximates the shifted operator T = alpha I - L by Xbar Theta
      // Xbar^T, Theta = alpha - nu.  The pairs are tracked in the L form, and alpha' I - H_T
      // with H_T = C Theta C^T + Z^T Delta_T Z, Delta_T = T' - pad(T), works out (Z^T Z = I) to
      //   C nu C^T + Z^T Delta_L Z + alpha (I - C C^T - Z_new^T Z_new),
      // Delta_L = L' - pad(L) the gathered product and Z_new the appended rows of Z: same
      // Ritz vectors, nu' = alpha' - theta.  F is free until the eigensolve: it holds the Gram.
      const int64_t s_new = n2 - st->n;
      if (s_new > 0)
        launch_tn<T, true>(s_new, b.Zc + (size_t)st->n * st->ldz, st->ldz, st->D, b.Zc + (size_t)st->n * st->ldz,
                           st->ldz, st->D, st->partial, st->F, st->stream);
      launch_lowrank_h(st->D, st->K, st->Clr, st->theta, st->H, st->stream, s_new > 0 ? st->F : nullptr,
                       st->maxdeg[st->gcur]);
    } else {
      launch_lowrank_h(st->D, st->K, st->Clr, st->theta, st->H, st->stream);
    }
  } else {
    // (op Z) with the updated operator (eq. RR_eigen_graph_upd_main2), L-form for Laplacians
    const int c0 = reuse ? st->K : 0;
    mark_spmm(st, 0);
    const HeavyRows hv = heavy_of(st, st->gcur ^ 1);  // the updated graph's buffer
    // the product covers the basis columns up to the padding of the row (columns the rest of
    // the update never reads), so that an odd width keeps 16-byte slices
    int wsp = st->D - c0;
    if (c0 % 4 == 0 && st->ldz % 4 == 0 && st->ldq == st->ldz) wsp = std::min(st->ldz - c0, (wsp + 3) / 4 * 4);
    launch_spmm<T>(st->op, n2, rp, col, sc, b.Zc + c0, st->ldz, n2, wsp, b.aux + c0, st->ldq, st->stream, &hv);
    mark_spmm(st, 1);
    st->spmm_cols[st->pslot] = st->D - c0;
    mark(st, 5);
    // H = Z^T (op Z)
    if constexpr (sizeof(T) == 4) {
      if (st->prec == GREST_MIXED)
        launch_tn_bf16(n2, b.Zc, st->ldz, st->D, b.aux, st->ldq, st->D, st->partial, st->H, st->stream);
      else
        launch_tn<T, false>(n2, b.Zc, st->ldz, st->D, b.aux, st->ldq, st->D, st->partial, st->H, st->stream);
    } else {
      launch_tn<T, true>(n2, b.Zc, st->ldz, st->D, b.aux, st->ldq, st->D, st->partial, st->H, st->stream);
    }
  }
  // small FP64 eigensolve on the leading K + rank block, selection of K pairs
  mark(st, 6);
  // with the overlap mode the next update's graph stage starts here: the one-workgroup
  // eigensolve leaves the rest of the device free for it
  if (gate_slot >= 0 && st->overlap && hipEventRecord(st->gate[gate_slot], st->stream) == hipSuccess)
    st->gate_recorded[gate_slot] = true;
  const int which = st->op == GREST_OP_ADJ ? 0 : 1;
  if (!small_eig_stage(st, st->D, base, rank_slot, st->H, which, st->K, 0.0, st->theta, st->F, nullptr, seg2,
                       rank2)) {
    snprintf(g_last_error, sizeof(g_last_error), "projected order %d outside the small eigensolver's range", st->D);
    return GREST_EINVAL;
  }
  // X' = Z F_K into the other buffer
  mark(st, 7);
  // X' = Z F on FP32 / FP64 MFMA (a memory-bound pass; FP32 keeps X orthonormal to 1e-7)
  launch_apply<T>(n2, b.Zc, st->ldz, st->D, st->F, st->K, 1.0, 0.0, b.Zn, st->ldz, st->stream);
  // A X' = (A Z) F, kept in aux[:, 0:K] for the next update (in place: every row of aux is
  // read before its first K entries are written)
  if (st->op == GREST_OP_ADJ && !lr)
    launch_apply<T>(n2, b.aux, st->ldq, st->D, st->F, st->K, 1.0, 0.0, b.aux, st->ldq, st->stream);
  mark(st, 8);
  return GREST_OK;
}

// The buffers an update sizes by its change list: the device copies of the change arrays,
// the packed keys of Delta before and after they are grouped by row, the insertion ranks
// of the merge, the ungrouped signs and the two slots of Delta's columns and signs.  grest_update uses the state's own (grown on demand), grest_update_noalloc
// those carved from the static device workspace.
struct ChangeBufs {
  int32_t *ei = nullptr, *ej = nullptr;
  int8_t* sg = nullptr;
  uint64_t *kin = nullptr, *kout = nullptr;
  int32_t* dcol[2] = {nullptr, nullptr};
  int8_t* dsg[2] = {nullptr, nullptr};
  int32_t* dins = nullptr;
  int8_t* sg_tmp = nullptr;
};

ChangeBufs state_change_bufs(const grest_state* st) {
  ChangeBufs b;
  b.ei = st->d_ei; b.ej = st->d_ej; b.sg = st->d_sg;
  b.kin = st->dkey_in; b.kout = st->dkey_out;
  for (int k = 0; k < 2; ++k) { b.dcol[k] = st->dcol[k]; b.dsg[k] = st->dsg[k]; }
  b.dins = st->dins; b.sg_tmp = st->dsg_tmp;
  return b;
}

// With ext the change-list buffers come from ext and nothing is allocated: the caller has
// checked every capacity the update needs.
template <typename T>
grest_status update_impl(grest_state* st, int64_t S, int64_t nc, const int32_t* ei, const int32_t* ej,
                         const int8_t* sg, const double* omega, int32_t where, const ChangeBufs* ext = nullptr) {
  hipStream_t s = st->stream;
  const int64_t n = st->n, n2 = n + S;
  // capacities
  if (!ext) {
    if (n2 > st->cap_n) CHK(grow_nodes(st, n2));
    if (!st->graph_free && st->m + 2 * nc > st->cap_m) CHK(grow_edges(st, st->m + 2 * nc));
    if (nc > st->cap_nc) CHK(alloc_change_arrays(st, std::max<int64_t>(nc, st->cap_nc * 2)));
    if (st->variant == GREST_RSVD && S > st->cap_s)
      CHK(alloc_sketch_arrays(st, std::max<int64_t>(S, 2 * st->cap_s)));
  }
  const ChangeBufs cb = ext ? *ext : state_change_bufs(st);
  // reuse of the kept A X (adjacency), with a full-width product every kAxRefresh updates
  // so that the rounding carried along by the recurrence stays bounded
  constexpr int kAxRefresh = 16;
  const bool lowrank = st->proj == GREST_PROJ_LOWRANK;
  const bool reuse = st->op == GREST_OP_ADJ && !lowrank && st->ax_valid && st->ax_age + 1 < kAxRefresh;

  const int gn = st->gcur ^ 1;
  const int ds = st->dslot;
  // ---- graph update and validation (Sec. 2, eq. adj_update) on the graph stream ----
  // It writes CSR buffer gn and Delta slot ds.  Without the overlap mode it simply
  // follows the earlier work on the one stream.  With it, it waits only for the last
  // readers of what it overwrites: the update two calls back, which used slot ds and
  // read buffer gn as its new graph; and the previous update, which read buffer gn as its
  // old graph in its own graph stage and, for the normalised Laplacian, in its Delta Xbar.
  // For the normalised Laplacian the stage starts once that Delta Xbar is done (ogate);
  // otherwise at the previous update's gate, recorded before its small eigensolve, which
  // also keeps this stage's many short kernels from queueing behind the wide ones before
  // it.  Without either event from the previous update (it stopped early) the stage waits
  // for that update's end, as it does after a rejected update, whose queued work reads the
  // scales of buffer gn.
  hipStream_t gs = st->gstream;
  st->gate_recorded[ds] = false;  // this update's events, once they are recorded
  st->ogate_recorded[ds] = false;
  if (gs != s) {
    if (st->end_recorded[ds]) HIPCHK(hipStreamWaitEvent(gs, st->endev[ds], 0));
    if (st->prev_rejected && st->end_recorded[ds ^ 1])
      HIPCHK(hipStreamWaitEvent(gs, st->endev[ds ^ 1], 0));
    else if (st->ogate_recorded[ds ^ 1])
      HIPCHK(hipStreamWaitEvent(gs, st->ogate[ds ^ 1], 0));
    else if (st->gate_recorded[ds ^ 1])
      HIPCHK(hipStreamWaitEvent(gs, st->gate[ds ^ 1], 0));
    else if (st->end_recorded[ds ^ 1])
      HIPCHK(hipStreamWaitEvent(gs, st->endev[ds ^ 1], 0));
  }
  const int32_t* dei = ei;
  const int32_t* dej = ej;
  const int8_t* dsgn = sg;
  if (where == GREST_HOST && nc > 0) {
    HIPCHK(hipMemcpyAsync(cb.ei, ei, nc * sizeof(int32_t), hipMemcpyHostToDevice, gs));
    HIPCHK(hipMemcpyAsync(cb.ej, ej, nc * sizeof(int32_t), hipMemcpyHostToDevice, gs));
    HIPCHK(hipMemcpyAsync(cb.sg, sg, nc * sizeof(int8_t), hipMemcpyHostToDevice, gs));
    dei = cb.ei; dej = cb.ej; dsgn = cb.sg;
  }
  int64_t* dptr = st->dptr[ds];
  int32_t* dcol = cb.dcol[ds];
  int8_t* dsg = cb.dsg[ds];
  int64_t* maxdeg = st->maxdeg[gn];
  st->marking = st->prof;
  mark(st, 0);
  launch_fill_bytes0(st->vstat[ds], sizeof(int32_t), gs);
  launch_fill_bytes0(maxdeg, sizeof(int64_t), gs);
  launch_fill_i64(st->dcnt, 0, n2 + 1, gs);
  const int kshift = delta_key_shift(n2);
  launch_delta_keys(dei, dej, dsgn, nc, n, S, kshift, cb.kin, cb.sg_tmp, st->dcnt, st->vstat[ds], gs);
  launch_scan_excl(st->dcnt, dptr, n2, st->scan_tmp, gs);
  // Delta's rows with more than HEAVY_DEG entries (only possible beyond HEAVY_DEG changes)
  const int64_t dh_bound = nc > HEAVY_DEG ? std::min<int64_t>(n2, 2 * nc / (HEAVY_DEG + 1) + 1) : 0;
  if (dh_bound > 0) launch_heavy_rows(n2, dptr, st->hflag, st->hpos, st->hscan, st->dhrows, st->dhcnt, gs);
  // the keys into their rows, each row sorted by column (the list of long rows uses the
  // new-length array, which the row pass below fills afterwards)
  launch_delta_group(cb.kin, cb.sg_tmp, 2 * nc, kshift, n2, dptr, st->dcnt, cb.kout, dsg, st->newlen, st->vstat[ds],
                     gs);
  launch_delta_extract(cb.kout, 2 * nc, dptr + n2, kshift, dcol, gs);
  const bool gfree = st->graph_free;
  launch_delta_rows(n, S, dptr, dcol, dsg, cb.dins, gfree ? nullptr : st->rp[st->gcur],
                    gfree ? nullptr : st->col[st->gcur], st->newlen, st->vstat[ds], gs);
  if (!gfree) {
    launch_scan_excl(st->newlen, st->rp[gn], n2, st->scan_tmp, gs);
    if (sizeof(T) == 8) launch_degrees(n2, st->rp[gn], (double*)st->sc[gn], nullptr, maxdeg, gs);
    else launch_degrees(n2, st->rp[gn], nullptr, (float*)st->sc[gn], maxdeg, gs);
    launch_heavy_rows(n2, st->rp[gn], st->hflag, st->hpos, st->hscan, st->hrows[gn], st->hcnt[gn], gs);
  }
  // ---- the work of the update that reads only Delta, the new graph's scales and Omega,
  // and writes only scratch (the sketch and the row lists), goes on the same stream, its
  // short kernels before the merge, which streams the whole graph ----
  const T* sc_new = (const T*)st->sc[gn];
  const bool nlap = st->op == GREST_OP_NLAP;
  const bool rsvd = st->variant == GREST_RSVD;
  const bool sparse_dx = !nlap && (rsvd || st->variant == GREST_G2);
  const int64_t sk_bound = std::min<int64_t>(n2, S + 2 * nc);
  if (rsvd && S > 0) {
    // S.1 (first half): Y = Delta_2 Omega; the projection comes with the orthonormalisation
    const int Ls = st->Ls;
    T* Y = (T*)st->ybuf;
    const double* om = omega;
    if (where == GREST_HOST) {
      HIPCHK(hipMemcpyAsync(st->omega64, omega, (size_t)S * Ls * sizeof(double), hipMemcpyHostToDevice, gs));
      om = st->omega64;
    }
    if (sizeof(T) == 8) {
      HIPCHK(hipMemcpyAsync(st->omega_t, om, (size_t)S * Ls * sizeof(double), hipMemcpyDeviceToDevice, gs));
    } else {
      launch_convert<double, float>(om, (float*)st->omega_t, (int64_t)S * Ls, gs);
    }
    // Y is zero except on the appended rows and the rows of Delta with an entry in an
    // appended column (the row list).  The buffer is kept that way: the rows of the
    // previous list are cleared (all of Y after a reallocation) and the product writes
    // the rows of the new list only.
    if (st->y_clean)
      launch_zero_listed_rows<T>(Y, st->ldy, Ls, st->srows, st->srows_cnt, st->srows_bound, gs);
    else
      launch_fill_rows<T>(Y, st->ldy, 0, n2, Ls, gs);
    launch_sketch_rows(n, S, dptr, dcol, st->rflag, st->rpos, st->rscan_tmp, st->srows, gs);
    launch_copy_i64(st->rpos + n2, st->srows_cnt, gs);
    st->srows_bound = sk_bound;
    st->y_clean = true;
    launch_delta_mul<T>(1, st->op, n, S, dptr, dcol, dsg, maxdeg, sc_new, (const T*)st->omega_t, Ls, Ls, Y,
                        st->ldy, gs, nullptr, 0, st->srows, st->rpos + n2, sk_bound);
  }
  // rows where Delta_1 X can be nonzero (the adjacency's and the Laplacian's form)
  if (sparse_dx || lowrank)
    launch_delta1_rows(n, S, dptr, dcol, st->dflag, st->dpos, st->dscan_tmp, st->drows, gs);
  if (!gfree)
    launch_csr_merge(n, S, st->rp[st->gcur], st->col[st->gcur], dptr, dcol, dsg, cb.dins, st->rp[gn], st->col[gn],
                     st->cap_m, gs);
  HIPCHK(hipMemcpyAsync(&st->pin->g[ds].vstatus, st->vstat[ds], sizeof(int32_t), hipMemcpyDeviceToHost, gs));
  if (!gfree) {
    HIPCHK(hipMemcpyAsync(&st->pin->g[ds].m_new, st->rp[gn] + n2, sizeof(int64_t), hipMemcpyDeviceToHost, gs));
    HIPCHK(hipMemcpyAsync(&st->pin->g[ds].hcount, st->hcnt[gn], sizeof(int64_t), hipMemcpyDeviceToHost, gs));
  }
  if (st->marking && st->stage_marks) (void)hipEventRecord(st->gend[st->pslot], gs);
  HIPCHK(hipEventRecord(st->gev[ds], gs));
  st->dslot ^= 1;
  // the rest of the update follows the graph stage; the numerical status word is cleared
  // for it (the previous update's word has been copied out by then, on this stream)
  if (gs != s) HIPCHK(hipStreamWaitEvent(s, st->gev[ds], 0));
  launch_fill_bytes0(st->status, sizeof(int32_t), s);
  // every return below records the end of this update's kernels (they read slot ds)
  struct EndMark {
    grest_state* st;
    int slot;
    ~EndMark() {
      if (hipEventRecord(st->endev[slot], st->stream) == hipSuccess) st->end_recorded[slot] = true;
    }
  } end_mark{st, ds};

  // The host needs the validation result before it commits.  Work that reads only the
  // update's own arrays (whose column ids are in range whatever the validation finds,
  // since out-of-range entries never enter them) and the current basis, and writes only
  // scratch blocks, is queued before the host waits for the validation event, so the
  // device keeps running meanwhile; a rejected update leaves nothing but scratch behind.
  // What reads the merged graph (the normalised Laplacian's Delta Xbar and the Rayleigh-
  // Ritz product) is queued after the wait.
  Blocks<T> b = blocks<T>(st);
  const int K = st->K;
  // Basis layout.  G-REST2/3: Z = [Xbar | Delta Xbar | augmentation], the last two
  // projected against Xbar and orthonormalised together.  RSVD: Z = [Xbar | R | Delta
  // Xbar]; the sketch basis R = M U_L is orthonormal and orthogonal to Xbar by
  // construction (M comes out of two projections and CholQR2, U_L is orthonormal), so
  // only Delta Xbar is projected, against [Xbar R], which spans the same subspace as
  // projecting [Delta Xbar, R] against Xbar (Sec. 3.5) with a third of the Gram work.
  T* dX = rsvd ? b.Zc + K + st->L : b.W;  // Delta Xbar
  T* Rb = b.Zc + K;                        // R (RSVD)
  // Delta Xbar is zero except on the rows of Delta with an entry in an old column (for the
  // adjacency and the Laplacian's form; the normalised Laplacian's form changes whole
  // rows), so the first projection round of a block made of it alone covers those rows
  auto project = [&]() {
    if (sparse_dx) {  // the row list came with the graph stage
      const int64_t bound = std::min<int64_t>(n2, 2 * nc);
      if (rsvd)
        orth_against<T>(st, n2, b.Zc, st->ldz, K + st->L, dX, st->ldz, K, 0, st->drows, st->dpos + n2, bound,
                        nullptr, st->dflag);
      else
        orth_against<T>(st, n2, b.Zc, st->ldz, K, b.W, st->ldz, st->Dw, 0, st->drows, st->dpos + n2, bound,
                        nullptr, st->dflag);
    } else if (rsvd) {
      orth_against<T>(st, n2, b.Zc, st->ldz, K + st->L, dX, st->ldz, K, 0);
    } else {
      orth_against<T>(st, n2, b.Zc, st->ldz, K, b.W, st->ldz, st->Dw, 0);
    }
  };
  // ---- pad Xbar (Alg. 2): zero the appended rows of the whole basis row ----
  mark(st, 1);
  launch_fill_rows<T>(b.Zc, st->ldz, n, S, st->ldz, s);
  // ---- Delta Xbar = Delta_1 X (Prop. 3) ----
  const HeavyRows dheavy{st->dhrows, st->dhcnt, dh_bound};
  if (sparse_dx) {
    // visit only the rows of Delta (the row list of the graph stage); the rest of the block
    // is zeroed first unless the projection's first round reads the listed rows alone (it
    // then writes the whole block)
    bool listed_only = false;
    if constexpr (sizeof(T) == 4) {
      listed_only = rsvd ? orth_reads_listed_rows_only(b.Zc, st->ldz, K + st->L, dX, st->ldz, K)
                         : orth_reads_listed_rows_only(b.Zc, st->ldz, K, b.W, st->ldz, st->Dw);
    }
    if (!listed_only) launch_fill_rows<T>(dX, st->ldz, 0, n2, K, s);
    if (reuse) launch_fill_rows<T>(b.aux, st->ldq, n, S, K, s);
    launch_delta_mul<T>(0, st->op, n, S, dptr, dcol, dsg, maxdeg, sc_new, b.Zc, st->ldz, K, dX, st->ldz, s,
                        reuse ? b.aux : nullptr, st->ldq, st->drows, st->dpos + n2, std::min<int64_t>(n2, 2 * nc),
                        &dheavy);
  } else if (!nlap) {
    launch_delta_mul<T>(0, st->op, n, S, dptr, dcol, dsg, maxdeg, sc_new, b.Zc, st->ldz, K, dX,
                        st->ldz, s, reuse ? b.aux : nullptr, st->ldq, nullptr, nullptr, 0, &dheavy);
  }
  st->ax_valid = false;  // valid again only once this update commits
  mark(st, 2);
  // ---- augmentation block ----
  if (st->variant == GREST_G3) {
    T* B2 = b.W + K;
    const int w2 = st->Dw - K;
    launch_fill_rows<T>(B2, st->ldz, 0, n2, w2, s);
    if (S > 0)
      launch_delta_mul<T>(3, st->op, n, S, dptr, dcol, dsg, maxdeg, sc_new, nullptr, 0, w2, B2,
                          st->ldz, s);
  } else if (rsvd) {
    if (S == 0) {
      launch_fill_rows<T>(Rb, st->ldz, 0, n2, st->L, s);
      launch_fill_bytes0(st->ranks + 4, sizeof(int32_t), s);  // no sketch columns kept
    } else {
      // S.1: Y = (I - Pi) Delta_2 Omega; Delta_2 Omega and its row list came with the
      // graph stage
      const int Ls = st->Ls;
      T* Mb = (T*)st->mbuf;
      const int64_t bound = sk_bound;
      // (I - Pi) applied twice and S.2: M = orth(Y), in the same two fused rounds; the first
      // round's read passes cover the listed rows of Y only, and its output Y1 goes to its
      // own buffer.  M = [Xbar Y1] Mchol is needed in full only through R = M U_L, so the
      // second round stops at its factor: M is formed on the listed rows alone (all that
      // Delta_2^T M reads; into Y's rows, which keeps Y zero elsewhere), and R comes out of
      // one pass over [Xbar Y1] with the coefficients Mchol U_L.
      orth_against<T>(st, n2, b.Zc, st->ldz, K, b.Y, st->ldy, Ls, 2, st->srows, st->rpos + n2, bound, Mb,
                      st->rflag, false);
      launch_apply2<T>(bound, b.Zc, st->ldz, K, Mb, st->ldy, Ls, st->Mchol, Ls, 1.0, 0.0, b.Y, st->ldy, s, nullptr,
                       st->srows, st->srows_cnt);
      const T* Mrows = b.Y;
      // B^T = Delta_2^T M; B B^T (FP64) and its leading eigenvectors U_L
      launch_delta_mul<T>(2, st->op, n, S, dptr, dcol, dsg, maxdeg, sc_new, Mrows, st->ldy, Ls,
                          (T*)st->bt, Ls, s, nullptr, 0, nullptr, nullptr, 0, &dheavy);
      launch_tn<T, true>(S, (const T*)st->bt, Ls, Ls, (const T*)st->bt, Ls, Ls, st->partial, st->Gm, s);
      if (!small_eig_stage(st, Ls, 0, st->ranks + 3, st->Gm, 2, st->L, st->tol, st->thetab, st->Fb,
                           st->ranks + 4)) {
        (void)hipEventSynchronize(st->gev[ds]);
        st->prev_rejected = true;  // nothing committed; queued work may still read slot ds
        st->marking = false;
        snprintf(g_last_error, sizeof(g_last_error), "sketch order %d outside the small eigensolver's range", Ls);
        return GREST_EINVAL;
      }
      // S.4: R = M U_L (its kept columns first, the dropped ones zero)
      launch_small_gemm(K + Ls, Ls, st->L, st->Mchol, st->Fb, st->Msk, s);
      launch_apply2<T>(n2, b.Zc, st->ldz, K, Mb, st->ldy, Ls, st->Msk, st->L, 1.0, 0.0, Rb, st->ldz, s);
    }
  }
  mark(st, 3);
  // ---- projection (I - Pi) twice and CholQR2 ----
  if (!nlap) project();

  HIPCHK(hipEventSynchronize(st->gev[ds]));
  // every earlier update has finished (with the overlap mode, once the previous update's
  // end event has passed): collect the numerical status and the stage times of the last one
  if (gs != s && st->end_recorded[ds ^ 1]) HIPCHK(hipEventSynchronize(st->endev[ds ^ 1]));
  st->deferred |= st->pin->status & ST_NUMERIC;
  st->pin->status = 0;
  prof_collect_slot(st, st->pslot ^ 1);
  const int32_t vbits = st->pin->g[ds].vstatus;
  st->prev_rejected = (vbits & VALIDATION_BITS) != 0;
  if (st->prev_rejected) {
    st->marking = false;
    snprintf(g_last_error, sizeof(g_last_error), "change list rejected (status bits 0x%x)", vbits);
    return GREST_EINVAL;
  }
  const int64_t m_new = gfree ? -1 : st->pin->g[ds].m_new;
  st->hcnt_host[gn] = gfree ? 0 : st->pin->g[ds].hcount;

  if (nlap) {
    const HeavyRows hv = heavy_of(st, gn);
    launch_nlap_delta_x<T>(n, S, st->rp[st->gcur], st->col[st->gcur], (const T*)st->sc[st->gcur], st->rp[gn],
                           st->col[gn], sc_new, b.Zc, st->ldz, K, dX, st->ldz, s, &hv);
    // the last read of the old graph (buffer gcur, which the next update's graph stage
    // overwrites); the rest of this update reads the new graph alone
    if (gs != s && hipEventRecord(st->ogate[ds], s) == hipSuccess) st->ogate_recorded[ds] = true;
    project();
  }
  mark(st, 4);
  // ---- Rayleigh-Ritz on Z = [Xbar, Q] and back-projection ----
  const LowRankIn lr_in{dptr, dcol, dsg, st->drows, st->dpos + n2, std::min<int64_t>(n2, 2 * nc)};
  const LowRankIn* lr = lowrank ? &lr_in : nullptr;
  if (rsvd)  // kept columns: [0, K + r_R) and [K + L, K + L + r_dX)
    CHK(rayleigh_ritz<T>(st, n2, st->rp[gn], st->col[gn], sc_new, K, st->ranks + 4, reuse, K + st->L, st->ranks + 1,
                         ds, lr));
  else
    CHK(rayleigh_ritz<T>(st, n2, st->rp[gn], st->col[gn], sc_new, K, st->ranks + 1, reuse, 0, nullptr, ds, lr));
  // status, ranks and the K Ritz values in one transfer (outbox mirrors Pinned from status on)
  HIPCHK(hipMemcpyAsync(&st->pin->status, st->outbox, OUT_HDR + st->K * sizeof(double), hipMemcpyDeviceToHost, s));
  // ---- commit ----
  if (st->marking) {  // the next update records into the other set
    st->prof_pending[st->pslot] = true;
    st->pslot ^= 1;
  }
  st->marking = false;
  st->gcur = gn;
  st->zcur ^= 1;
  st->n = n2;
  st->m = m_new;
  st->ax_valid = st->op == GREST_OP_ADJ && !lowrank;
  st->ax_age = reuse ? st->ax_age + 1 : 0;
  return GREST_OK;
}


// Default residual tolerance of the initial eigensolver: max_j ||M x_j - lambda_j x_j|| /
// scale (scale as for the drift measure), near what the precision of the blocks can reach.
double default_init_tol(const grest_state* st) { return st->es == 8 ? 1e-12 : 4e-6; }

// Initial pairs (Alg. 2 line 3, "any direct eigendecomposition method"): a Chebyshev-
// filtered block subspace iteration on the tracked operator, with Rayleigh-Ritz after
// every filter and a residual stop.  The block has b = min(D, 128, n) columns (D the
// basis width, at least K).  Starting from a random block orthonormalised by CholQR2,
// each outer step
//  1. runs Rayleigh-Ritz on the orthonormal block Z: (op Z) by the sparse product, H =
//     Z^T (op Z) with FP64 accumulation, all b Ritz pairs by the small FP64 eigensolver
//     in the order of the selection (largest magnitude for the adjacency; smallest nu for
//     the Laplacians, whose products are taken in the L-form), X = Z F and (op X) =
//     (op Z) F;
//  2. measures the residual of the K leading pairs, max_j ||(op) x_j - theta_j x_j|| /
//     scale with scale = max_j |theta_j| (adjacency), 2 d_max (L) or 2 (L_n), and stops
//     when it is at most tol or the product budget is spent;
//  3. filters the Ritz block by the Chebyshev polynomial T_m of the operator mapped so
//     that the interval of the unwanted spectrum becomes [-1, 1]: [-c, c] with c the
//     smallest magnitude in the block (adjacency), [nu_b, 2 d_max] or [nu_b, 2] with nu_b
//     the largest nu in the block (Laplacians; both bound the spectrum of L and L_n from
//     above).  The degree m is the largest whose growth at the block's leading Ritz value
//     stays below 1e4, so that CholQR2 of the filtered block stays well conditioned (at
//     most 16, at least 1); T_m comes from the three-term recurrence
//     Y_{j+1} = (2/e)(op Y_j - center Y_j) - Y_{j-1}; then CholQR2.
// The pairs of the last Rayleigh-Ritz step are committed; *products and *resid report
// the products with the operator used and the last residual.
template <typename T>
grest_status init_impl(grest_state* st, int max_products, double tol, uint64_t seed, int32_t* products_out,
                       double* resid_out) {
  hipStream_t s = st->stream;
  const int64_t n = st->n;
  const int K = st->K;
  int b = std::min(st->D, 128);
  if (b > n) b = (int)n;
  if (b < K || max_products < 1) return GREST_EINVAL;
  const bool adj = st->op == GREST_OP_ADJ;
  const int which = adj ? 0 : 1;
  T* buf[2] = {(T*)st->z[0], (T*)st->z[1]};
  int cur = st->zcur;  // buffer of the orthonormal block
  T* aux = (T*)st->aux;
  const int64_t* rp = st->rp[st->gcur];
  const int32_t* col = st->col[st->gcur];
  const T* sc = (const T*)st->sc[st->gcur];
  const HeavyRows hv = heavy_of(st, st->gcur);
  double hi = 0.0;  // upper bound of the spectrum of L (2 d_max) or L_n (2)
  if (st->op == GREST_OP_LAP) {
    int64_t md = 0;
    HIPCHK(hipMemcpy(&md, st->maxdeg[st->gcur], sizeof(int64_t), hipMemcpyDeviceToHost));
    hi = 2.0 * (double)md;
  } else if (st->op == GREST_OP_NLAP) {
    hi = 2.0;
  }
  launch_fill_bytes0(st->status, sizeof(int32_t), s);
  launch_fill_rows<T>(buf[cur], st->ldz, 0, n, st->ldz, s);
  launch_fill_random<T>(buf[cur], st->ldz, n, b, seed, s);
  cholqr2<T>(st, n, buf[cur], st->ldz, b, 0);
  std::vector<double> th((size_t)b), gram((size_t)K * K);
  int32_t rk[8] = {};
  int products = 0;
  double resid = INFINITY;
  for (;;) {
    T* Z = buf[cur];
    T* X = buf[cur ^ 1];
    // 1. Rayleigh-Ritz on Z (its kept columns)
    launch_spmm<T>(st->op, n, rp, col, sc, Z, st->ldz, n, b, aux, st->ldq, s, &hv);
    ++products;
    launch_tn<T, true>(n, Z, st->ldz, b, aux, st->ldq, b, st->partial, st->H, s);
    launch_symmetrize(b, st->H, s);
    if (!launch_small_eig(b, 0, st->ranks + 1, st->H, which, b, 0.0, st->theta, st->F, nullptr, st->eigwork,
                          st->status, s)) {
      snprintf(g_last_error, sizeof(g_last_error), "initial block width %d outside the small eigensolver's range", b);
      return GREST_EINVAL;
    }
    launch_apply<T>(n, Z, st->ldz, b, st->F, b, 1.0, 0.0, X, st->ldz, s);
    launch_apply<T>(n, aux, st->ldq, b, st->F, b, 1.0, 0.0, aux, st->ldq, s);  // (op X), in place
    // 2. residual block of the K leading pairs, in Z's buffer (free from here on)
    launch_lincomb3<T>(n, K, 1.0, aux, st->ldq, 0.0, aux, st->ldq, 0.0, nullptr, 0, Z, st->ldz, s);
    launch_sub_scaled_cols<T>(n, K, st->theta, X, st->ldz, Z, st->ldz, s);
    launch_tn<T, true>(n, Z, st->ldz, K, Z, st->ldz, K, st->partial, st->Gm, s);
    HIPCHK(hipMemcpyAsync(gram.data(), st->Gm, gram.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(th.data(), st->theta, th.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(rk, st->ranks, sizeof(rk), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&st->pin->status, st->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    cur ^= 1;  // the Ritz block X is the current block
    if (st->pin->status & ST_NUMERIC) break;
    double scale = hi;
    if (adj) {
      scale = 0.0;
      for (int j = 0; j < K; ++j) scale = std::max(scale, std::fabs(th[(size_t)j]));
    }
    if (!(scale > 0.0)) scale = 1.0;
    double m2 = 0.0;
    for (int j = 0; j < K; ++j) m2 = std::max(m2, gram[(size_t)j * K + j]);
    resid = std::sqrt(m2) / scale;
    if (resid <= tol || max_products - products < 2) break;
    // 3. Chebyshev filter of the Ritz block (its nb valid columns, ordered by the selection)
    const int nb = std::max(1, std::min(b, (int)rk[1]));
    double center, e, r0;
    if (adj) {
      double c = std::fabs(th[(size_t)nb - 1]);
      if (!(c > 0.0)) c = 0.5 * std::fabs(th[0]);
      center = 0.0;
      e = c > 0.0 ? c : 1.0;
      r0 = std::fabs(th[0]) / e;
    } else {
      const double lo = th[(size_t)nb - 1];
      const double top = std::max(hi, lo + 1e-12 * std::max(1.0, hi));
      center = 0.5 * (lo + top);
      e = 0.5 * (top - lo);
      r0 = (center - th[0]) / e;
    }
    int m = 1;
    if (r0 > 1.0 + 1e-12) m = (int)std::floor(std::acosh(1e4) / std::acosh(r0));
    m = std::max(1, std::min(m, std::min(16, max_products - products - 1)));
    T* prev = buf[cur];
    T* next = buf[cur ^ 1];
    launch_spmm<T>(st->op, n, rp, col, sc, prev, st->ldz, n, b, aux, st->ldq, s, &hv);
    ++products;
    launch_lincomb3<T>(n, b, 1.0 / e, aux, st->ldq, -center / e, prev, st->ldz, 0.0, nullptr, 0, next, st->ldz, s);
    for (int j = 1; j < m; ++j) {
      launch_spmm<T>(st->op, n, rp, col, sc, next, st->ldz, n, b, aux, st->ldq, s, &hv);
      ++products;
      // T_{j+1} into the buffer of T_{j-1} (element by element, read before written)
      launch_lincomb3<T>(n, b, 2.0 / e, aux, st->ldq, -2.0 * center / e, next, st->ldz, -1.0, prev, st->ldz, prev,
                         st->ldz, s);
      std::swap(prev, next);
    }
    cur = next == buf[0] ? 0 : 1;
    cholqr2<T>(st, n, buf[cur], st->ldz, b, 0);
  }
  HIPCHK(hipMemcpyAsync(st->theta_pin, st->theta, st->K * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  st->zcur = cur;
  st->has_pairs = true;
  st->ax_valid = st->op == GREST_OP_ADJ && st->proj == GREST_PROJ_EXACT;  // aux[:, 0:K] = A X
  st->ax_age = 0;
  st->rs_since_check = st->rs_since_start = 0;
  st->last_init_products = products;
  st->last_init_resid = resid;
  if (products_out) *products_out = products;
  if (resid_out) *resid_out = resid;
  if (st->pin->status & ST_NUMERIC) return GREST_ENUMERIC;
  return GREST_OK;
}

// Drift of the tracked pairs (the measure a restart is decided on): orth = max |U^T U - I|
// and resid = max_j ||M u_j - lambda_j u_j||_2 / scale, with M the matrix whose values are
// reported (A, L or L_n) and scale = max_j |lambda_j| (adjacency), 2 d_max (L) or 2 (L_n),
// the bounds on their norms of Sec. 4.2.  Gram and residual norms accumulate in FP64; the
// residual block M U - U diag(lambda) is formed in the other basis buffer, which is scratch
// between updates.  Without a stored graph resid is NaN.
template <typename T>
grest_status drift_impl(grest_state* st, double* orth, double* resid) {
  CHK(sync_all(st));
  hipStream_t s = st->stream;
  const int64_t n = st->n;
  const int K = st->K;
  const T* U = (const T*)st->z[st->zcur];
  T* R = (T*)st->z[st->zcur ^ 1];
  launch_tn<T, true>(n, U, st->ldz, K, U, st->ldz, K, st->partial, st->Gm, s);
  std::vector<double> G((size_t)K * K), RR((size_t)K * K);
  HIPCHK(hipMemcpyAsync(G.data(), st->Gm, G.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  int64_t md = 0;
  if (!st->graph_free) {
    const HeavyRows hv = heavy_of(st, st->gcur);
    launch_spmm<T>(st->op, n, st->rp[st->gcur], st->col[st->gcur], (const T*)st->sc[st->gcur], U, st->ldz, n, K, R,
                   st->ldz, s, &hv);
    launch_sub_scaled_cols<T>(n, K, st->theta, U, st->ldz, R, st->ldz, s);
    launch_tn<T, true>(n, R, st->ldz, K, R, st->ldz, K, st->partial, st->H, s);
    HIPCHK(hipMemcpyAsync(RR.data(), st->H, RR.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&md, st->maxdeg[st->gcur], sizeof(int64_t), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  double o = 0.0;
  for (int i = 0; i < K; ++i)
    for (int j = 0; j < K; ++j) o = std::max(o, std::fabs(G[(size_t)i * K + j] - (i == j ? 1.0 : 0.0)));
  double r = std::nan("");
  if (!st->graph_free) {
    double scale = 0.0;
    if (st->op == GREST_OP_ADJ) {
      for (int j = 0; j < K; ++j) scale = std::max(scale, std::fabs(st->theta_pin[j]));
    } else {
      scale = st->op == GREST_OP_LAP ? 2.0 * (double)md : 2.0;
    }
    if (!(scale > 0.0)) scale = 1.0;
    double m2 = 0.0;
    for (int j = 0; j < K; ++j) m2 = std::max(m2, RR[(size_t)j * K + j]);
    r = std::sqrt(m2) / scale;
  }
  if (orth) *orth = o;
  if (resid) *resid = r;
  return GREST_OK;
}

bool host_changes_ok(int64_t n, int64_t S, int64_t nc, const int32_t* ei, const int32_t* ej, const int8_t* sg) {
  if (nc < 0 || S < 0) return false;
  if (nc == 0) return true;
  if (!ei || !ej || !sg) return false;
  const int64_t n2 = n + S;
  std::vector<int64_t> keys((size_t)nc);
  for (int64_t c = 0; c < nc; ++c) {
    const int64_t i = ei[c], j = ej[c];
    const int s = sg[c];
    if (i < 0 || j <= i || j >= n2) return false;
    if (s != 1 && s != -1) return false;
    if (j >= n && s != 1) return false;
    keys[(size_t)c] = i * n2 + j;
  }
  std::sort(keys.begin(), keys.end());
  return std::adjacent_find(keys.begin(), keys.end()) == keys.end();
}

template <typename T>
grest_status set_pairs_impl(grest_state* st, const double* values, const double* X, int32_t where) {
  const int64_t n = st->n;
  const int K = st->K;
  hipStream_t s = st->stream;
  const size_t cnt = (size_t)n * K;
  double* tmp = nullptr;
  CHK(dalloc(&tmp, cnt));
  if (where == GREST_HOST) {
    HIPCHK(hipMemcpyAsync(tmp, X, cnt * sizeof(double), hipMemcpyHostToDevice, s));
  } else {
    HIPCHK(hipMemcpyAsync(tmp, X, cnt * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  T* Z = (T*)st->z[st->zcur];
  T* packed = (T*)st->z[st->zcur ^ 1];  // the other basis buffer is scratch between updates
  if (sizeof(T) == 8) HIPCHK(hipMemcpyAsync(packed, tmp, cnt * sizeof(double), hipMemcpyDeviceToDevice, s));
  else launch_convert<double, float>(tmp, (float*)packed, (int64_t)cnt, s);
  HIPCHK(hipMemcpy2DAsync(Z, st->ldz * sizeof(T), packed, K * sizeof(T), K * sizeof(T), n, hipMemcpyDeviceToDevice, s));
  if (where == GREST_HOST) {
    memcpy(st->theta_pin, values, K * sizeof(double));
  } else {
    HIPCHK(hipMemcpyAsync(st->theta_pin, values, K * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemcpy(st->theta, st->theta_pin, K * sizeof(double), hipMemcpyHostToDevice));
  dfree(tmp);
  st->has_pairs = true;
  st->ax_valid = false;
  st->rs_since_check = st->rs_since_start = 0;
  return GREST_OK;
}

template <typename T>
grest_status get_impl(grest_state* st, double* values, void* X, int32_t x_dtype, int32_t where) {
  hipStream_t s = st->stream;
  HIPCHK(hipStreamSynchronize(s));
  if (values) memcpy(values, st->theta_pin, st->K * sizeof(double));
  if (!X) return GREST_OK;
  const int64_t n = st->n;
  const int K = st->K;
  const T* Z = (const T*)st->z[st->zcur];
  T* packed = (T*)st->z[st->zcur ^ 1];  // scratch between updates (the product buffer is kept)
  HIPCHK(hipMemcpy2DAsync(packed, K * sizeof(T), Z, st->ldz * sizeof(T), K * sizeof(T), n, hipMemcpyDeviceToDevice, s));
  const size_t cnt = (size_t)n * K;
  const void* src = packed;
  size_t bytes = cnt * sizeof(T);
  void* conv = nullptr;
  if ((x_dtype == GREST_F64) != (sizeof(T) == 8)) {
    if (x_dtype == GREST_F64) {
      double* c = nullptr;
      CHK(dalloc(&c, cnt));
      launch_convert<float, double>((const float*)packed, c, (int64_t)cnt, s);
      conv = c; bytes = cnt * sizeof(double);
    } else {
      float* c = nullptr;
      CHK(dalloc(&c, cnt));
      launch_convert<double, float>((const double*)packed, c, (int64_t)cnt, s);
      conv = c; bytes = cnt * sizeof(float);
    }
    src = conv;
  }
  HIPCHK(hipMemcpyAsync(X, src, bytes, where == GREST_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  if (conv) (void)hipFree(conv);
  return GREST_OK;
}

}  // namespace

// Device bytes of the capacity-sized buffers at the given capacities (the sizes the
// allocation functions above request; the small fixed matrices are left out, they never
// grow).  The allocator may round each request up a little.
int64_t state_bytes_for(const grest_state* st, const StateCaps& c) {
  const int64_t es = (int64_t)st->es;
  const int64_t n1 = c.cap_n + 1;
  int64_t b = 0;
  b += 2 * n1 * 8 + 2 * c.cap_n * es + 2 * c.cap_n * st->ldz * es;  // rp, sc, z (two each)
  if (!st->graph_free) b += c.cap_n * st->ldq * es;  // (op Z)
  if (st->variant == GREST_RSVD) b += 2 * c.cap_n * st->ldy * es;    // sketch and its basis
  b += 10 * n1 * 8;                                                  // counts, offsets, flags, positions
  b += 4 * (scan_tmp_elems(n1) + 16) * 8;                            // scan workspaces
  b += 5 * n1 * 4;                                                   // row lists
  if (!st->graph_free) b += 2 * c.cap_m * 4;                         // column ids (two buffers)
  const int64_t nc = c.cap_nc;
  b += nc * (4 + 4 + 1) + 2 * nc * (8 + 8 + 2 * 4 + 2 * 1 + 4 + 1);  // change arrays
  if (st->proj == GREST_PROJ_LOWRANK)
    b += 2 * std::max<int64_t>(1, std::min<int64_t>(2 * nc, c.cap_n)) * st->D * es;
  if (st->variant == GREST_RSVD) b += c.cap_s * st->Ls * (2 * es + 8);
  return b;
}

void state_caps(const grest_state* st, StateCaps* c) {
  c->cap_n = st->cap_n;
  c->cap_m = st->cap_m;
  c->cap_nc = st->cap_nc;
  c->cap_s = st->cap_s;
  c->n = st->n;
  c->m = st->m;
}

// The capacities after one more update of n_new nodes and nc changes, by the growth rule
// of the update (node and entry buffers by 1.5x, change and sketch buffers by 2x).
void state_caps_after(const grest_state* st, StateCaps* c, int64_t n_new, int64_t nc, int64_t dm) {
  const int64_t n2 = c->n + n_new;
  if (n2 > c->cap_n) c->cap_n = std::max<int64_t>(n2, c->cap_n + c->cap_n / 2);
  if (!st->graph_free && c->m + 2 * nc > c->cap_m) c->cap_m = std::max<int64_t>(c->m + 2 * nc, c->cap_m + c->cap_m / 2);
  if (nc > c->cap_nc) c->cap_nc = std::max<int64_t>(nc, c->cap_nc * 2);
  if (st->variant == GREST_RSVD && n_new > c->cap_s) c->cap_s = std::max<int64_t>(n_new, 2 * c->cap_s);
  c->n = n2;
  if (!st->graph_free) c->m += dm;
}

void* state_user_stream(const grest_state* st) { return st->own_stream ? nullptr : (void*)st->stream; }
int64_t state_sketch_cols(const grest_state* st) { return st->variant == GREST_RSVD ? st->Ls : 0; }
void state_rebind_stream(grest_state* st, void* stream) {
  st->stream = (hipStream_t)stream;
  if (!st->overlap) st->gstream = st->stream;
}

// =====================================================================================
// C interface
// =====================================================================================
extern "C" {

int32_t grest_abi_version(void) { return 1; }

const char* grest_strerror(grest_status status) {
  switch (status) {
    case GREST_OK: return "ok";
    case GREST_EINVAL: return "invalid argument or change list";
    case GREST_ENOMEM: return "out of memory";
    case GREST_EDEVICE: return "device error";
    case GREST_ENUMERIC: return "numerical failure";
    case GREST_ENODEV: return "no usable device";
    case GREST_EAGAIN: return "queue full or memory budget exceeded";
  }
  return "unknown status";
}

const char* grest_last_error(void) { return g_last_error; }

grest_status grest_validate_changes(int64_t n, int64_t n_new, int64_t n_changes, const int32_t* ei,
                                    const int32_t* ej, const int8_t* sign) {
  if (n < 0) return GREST_EINVAL;
  return host_changes_ok(n, n_new, n_changes, ei, ej, sign) ? GREST_OK : GREST_EINVAL;
}

namespace {
// exact_caps: the capacities are taken as given (a resumed checkpoint, whose later growth
// must happen at the same updates as the saved state's); otherwise they are lower bounds
grest_status create_impl(const grest_config* cfg, void* stream, int64_t n0, const int64_t* rowptr,
                         const int32_t* col, int64_t node_capacity, int64_t nnz_capacity, bool exact_caps,
                         grest_state** out) {
  if (!out) return GREST_EINVAL;
  *out = nullptr;
  if (!cfg || !rowptr || n0 < 1 || (n0 >= INT32_MAX)) return GREST_EINVAL;
  if (cfg->k < 1 || cfg->k >= n0 + (cfg->variant == GREST_G2 ? 0 : 0)) return GREST_EINVAL;
  if (cfg->k > 128) return GREST_EINVAL;
  if (cfg->variant != GREST_G2 && cfg->variant != GREST_G3 && cfg->variant != GREST_RSVD) return GREST_EINVAL;
  if (cfg->op < GREST_OP_ADJ || cfg->op > GREST_OP_NLAP) return GREST_EINVAL;
  if (cfg->precision < GREST_FP64 || cfg->precision > GREST_MIXED) return GREST_EINVAL;
  if (cfg->variant == GREST_RSVD && (cfg->L < 1 || cfg->P < 0 || cfg->L + cfg->P > 128)) return GREST_EINVAL;
  if (cfg->variant == GREST_G3 && cfg->max_new < 0) return GREST_EINVAL;
  if (cfg->proj != GREST_PROJ_EXACT && cfg->proj != GREST_PROJ_LOWRANK) return GREST_EINVAL;
  if (cfg->proj == GREST_PROJ_LOWRANK && cfg->op == GREST_OP_NLAP) return GREST_EINVAL;
  const int64_t m0 = rowptr[n0];
  if (m0 < 0 || (m0 > 0 && !col)) return GREST_EINVAL;
  // host check of the initial CSR: monotone offsets, ids in range, sorted, no self-loops
  for (int64_t r = 0; r < n0; ++r) {
    if (rowptr[r + 1] < rowptr[r] || rowptr[0] != 0) return GREST_EINVAL;
    for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      if (col[e] < 0 || col[e] >= n0 || col[e] == r) return GREST_EINVAL;
      if (e > rowptr[r] && col[e] <= col[e - 1]) return GREST_EINVAL;
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return GREST_ENODEV;

  grest_state* st = new (std::nothrow) grest_state();
  if (!st) return GREST_ENOMEM;
  st->cfg = *cfg;
  (void)hipGetDevice(&st->device);
  st->prec = cfg->precision;
  st->proj = cfg->proj;
  st->es = cfg->precision == GREST_FP64 ? 8 : 4;
  st->K = cfg->k;
  st->op = cfg->op;
  st->variant = cfg->variant;
  st->L = cfg->variant == GREST_RSVD ? cfg->L : 0;
  st->Ls = cfg->variant == GREST_RSVD ? cfg->L + cfg->P : 0;
  const int extra = cfg->variant == GREST_G3 ? cfg->max_new : (cfg->variant == GREST_RSVD ? cfg->L : 0);
  st->Dw = st->K + extra;
  st->D = st->K + st->Dw;
  // widths the kernels hold: every block orthonormalised by CholQR2 at most 128 columns
  // (the Cholesky factor; RSVD: Delta Xbar and the sketch, else the whole augmentation),
  // the basis at most 196 (the small eigensolver)
  const int orth_w = st->variant == GREST_RSVD ? std::max(st->K, st->Ls) : st->Dw;
  if (orth_w > 128 || st->D > 196) { delete st; return GREST_EINVAL; }
  const int q = (int)(16 / st->es);
  st->ldz = (int)round_up(st->D, q);
  st->ldq = st->ldz;
  st->ldy = (int)round_up(std::max(st->Ls, 1), q);
  st->tol = cfg->rank_tol > 0 ? cfg->rank_tol : (cfg->precision == GREST_FP64 ? 1e-7 : 1e-5);
  if (stream) {
    st->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&st->stream, hipStreamNonBlocking) != hipSuccess) { delete st; return GREST_EDEVICE; }
    st->own_stream = true;
  }
  st->gstream = st->stream;
  grest_status rc = GREST_OK;
  auto fail = [&](grest_status e) { free_all(st); if (st->own_stream) (void)hipStreamDestroy(st->stream); delete st; return e; };
  int64_t capn = exact_caps ? node_capacity : std::max<int64_t>(node_capacity, n0 + 1);
  if (capn < n0 || capn >= INT32_MAX) return fail(GREST_EINVAL);  // node ids are int32
  int64_t capm = exact_caps ? std::max<int64_t>(nnz_capacity, 1) : std::max<int64_t>(nnz_capacity, m0 + 1024);
  if (capm < m0) return fail(GREST_EINVAL);
  if ((rc = alloc_node_arrays(st, capn)) != GREST_OK) return fail(rc);
  if ((rc = alloc_edge_arrays(st, capm)) != GREST_OK) return fail(rc);
  // Room for a change list of 1/32 of the stored entries and for n0/64 nodes appended at
  // once, so that the first updates of a stream do not reallocate these arrays (each
  // reallocation drains the state's streams).  A low-rank state keeps two gathered basis
  // rows per change, so it starts small and grows on demand.
  const bool small_caps = exact_caps || cfg->proj == GREST_PROJ_LOWRANK;
  const int64_t cap_nc0 = small_caps ? 4096 : std::max<int64_t>(4096, m0 / 32);
  const int64_t cap_s0 = exact_caps ? 1024 : std::max<int64_t>(1024, n0 / 64);
  if ((rc = alloc_change_arrays(st, cap_nc0)) != GREST_OK) return fail(rc);
  if ((rc = alloc_sketch_arrays(st, cap_s0)) != GREST_OK) return fail(rc);
  const int dmax = st->D;
  const int wmax = std::max(st->Dw, std::max(st->Ls, 1));
  if ((rc = dalloc(&st->C1, (size_t)st->K * wmax)) != GREST_OK) return fail(rc);
  if ((rc = dalloc(&st->C2, (size_t)st->K * wmax)) != GREST_OK) return fail(rc);
  // the Gram and the factor also serve the initial eigensolver's blocks of up to D columns
  const size_t gw = (size_t)std::max(wmax, dmax);
  if ((rc = dalloc(&st->Gm, gw * gw)) != GREST_OK) return fail(rc);
  if ((rc = dalloc(&st->Mchol, std::max((size_t)(st->K + wmax) * wmax + (size_t)(wmax + 1) * (wmax + 1),
                                        gw * gw))) != GREST_OK)
    return fail(rc);
  if ((rc = dalloc(&st->M1buf, (size_t)(st->D + wmax) * wmax)) != GREST_OK) return fail(rc);
  if ((rc = dalloc(&st->Clr, (size_t)st->D * st->K)) != GREST_OK) return fail(rc);
  if ((rc = dalloc(&st->H, (size_t)dmax * dmax)) != GREST_OK) return fail(rc);
  if ((rc = dalloc(&st->Msk, (size_t)(st->K + wmax) * std::max(st->L, 1))) != GREST_OK) return fail(rc);
  // F and theta hold all the pairs of a block of the initial eigensolver (up to D)
  if ((rc = dalloc(&st->F, (size_t)dmax * dmax)) != GREST_OK) return fail(rc);
  if ((rc = dalloc((char**)&st->outbox, OUT_HDR + (size_t)dmax * sizeof(double))) != GREST_OK) return fail(rc);
  st->status = reinterpret_cast<int32_t*>(st->outbox);
  st->ranks = st->status + 1;
  st->theta = reinterpret_cast<double*>(static_cast<char*>(st->outbox) + OUT_HDR);
  if ((rc = dalloc(&st->Fb, (size_t)std::max(st->Ls, 1) * std::max(st->L, 1))) != GREST_OK) return fail(rc);
  if ((rc = dalloc(&st->thetab, std::max(st->L, 1))) != GREST_OK) return fail(rc);
  st->partial_elems = (int64_t)tn_num_chunks(INT64_MAX / 4) * dmax * dmax;
  if ((rc = dalloc(&st->partial, st->partial_elems)) != GREST_OK) return fail(rc);
  const int64_t ework = std::max(eig_work_elems(std::max(dmax, std::max(st->Ls, 1))), pchol_work_elems(wmax, st->K));
  if ((rc = dalloc(&st->eigwork, ework)) != GREST_OK) return fail(rc);
  if ((rc = dalloc(&st->dhcnt, 1)) != GREST_OK) return fail(rc);
  for (int b = 0; b < 2; ++b) {
    if ((rc = dalloc(&st->hcnt[b], 1)) != GREST_OK) return fail(rc);
    if ((rc = dalloc(&st->maxdeg[b], 1)) != GREST_OK) return fail(rc);
    if ((rc = dalloc(&st->vstat[b], 1)) != GREST_OK) return fail(rc);
    if (hipEventCreateWithFlags(&st->gev[b], hipEventDisableTiming) != hipSuccess) return fail(GREST_EDEVICE);
    if (hipEventCreateWithFlags(&st->endev[b], hipEventDisableTiming) != hipSuccess) return fail(GREST_EDEVICE);
    if (hipEventCreateWithFlags(&st->gate[b], hipEventDisableTiming) != hipSuccess) return fail(GREST_EDEVICE);
    if (hipEventCreateWithFlags(&st->ogate[b], hipEventDisableTiming) != hipSuccess) return fail(GREST_EDEVICE);
  }
  if ((rc = dalloc(&st->srows_cnt, 1)) != GREST_OK) return fail(rc);
  if (hipHostMalloc((void**)&st->pin, sizeof(Pinned) + (size_t)st->K * sizeof(double)) != hipSuccess)
    return fail(GREST_ENOMEM);
  st->theta_pin = reinterpret_cast<double*>(st->pin + 1);
  memset(st->pin, 0, sizeof(Pinned) + (size_t)st->K * sizeof(double));
  // upload the graph
  st->n = n0;
  st->m = m0;
  if (hipMemcpyAsync(st->rp[0], rowptr, (n0 + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st->stream) != hipSuccess)
    return fail(GREST_EDEVICE);
  if (m0 > 0 && hipMemcpyAsync(st->col[0], col, m0 * sizeof(int32_t), hipMemcpyHostToDevice, st->stream) != hipSuccess)
    return fail(GREST_EDEVICE);
  launch_fill_bytes0(st->maxdeg[0], sizeof(int64_t), st->stream);
  if (st->es == 8) launch_degrees(n0, st->rp[0], (double*)st->sc[0], nullptr, st->maxdeg[0], st->stream);
  else launch_degrees(n0, st->rp[0], nullptr, (float*)st->sc[0], st->maxdeg[0], st->stream);
  if ((rc = heavy_rows_sync(st, 0)) != GREST_OK) return fail(rc);
  // symmetry check on the device would need a transpose; the host check above covers format
  if (hipStreamSynchronize(st->stream) != hipSuccess) return fail(GREST_EDEVICE);
  *out = st;
  return GREST_OK;
}
}  // namespace

grest_status grest_create(const grest_config* cfg, void* stream, int64_t n0, const int64_t* rowptr,
                          const int32_t* col, int64_t node_capacity, int64_t nnz_capacity, grest_state** out) {
  return create_impl(cfg, stream, n0, rowptr, col, node_capacity, nnz_capacity, false, out);
}

grest_status grest_set_pairs(grest_state* st, const double* values, const double* X, int32_t where) {
  if (!st || !values || !X) return GREST_EINVAL;
  return st->es == 8 ? set_pairs_impl<double>(st, values, X, where) : set_pairs_impl<float>(st, values, X, where);
}

grest_status grest_init_pairs(grest_state* st, int32_t iterations, uint64_t seed) {
  if (!st || iterations < 1 || st->graph_free) return GREST_EINVAL;
  const double tol = default_init_tol(st);
  return st->es == 8 ? init_impl<double>(st, iterations, tol, seed, nullptr, nullptr)
                     : init_impl<float>(st, iterations, tol, seed, nullptr, nullptr);
}

grest_status grest_init_pairs_tol(grest_state* st, int32_t max_products, double tol, uint64_t seed,
                                  int32_t* products, double* resid) {
  if (!st || max_products < 1 || st->graph_free || !(tol >= 0.0)) return GREST_EINVAL;
  return st->es == 8 ? init_impl<double>(st, max_products, tol, seed, products, resid)
                     : init_impl<float>(st, max_products, tol, seed, products, resid);
}

grest_status grest_init_stats(const grest_state* st, int32_t* products, double* resid) {
  if (!st) return GREST_EINVAL;
  if (products) *products = st->last_init_products;
  if (resid) *resid = st->last_init_resid;
  return GREST_OK;
}

grest_status grest_update(grest_state* st, int64_t n_new, int64_t n_changes, const int32_t* ei, const int32_t* ej,
                          const int8_t* sign, const double* omega, int32_t where) {
  if (!st || !st->has_pairs) return GREST_EINVAL;
  if (n_new < 0 || n_changes < 0) return GREST_EINVAL;
  if (st->n + n_new >= INT32_MAX) return GREST_EINVAL;
  if (n_changes > 0 && (!ei || !ej || !sign)) return GREST_EINVAL;
  if (st->variant == GREST_G3 && n_new > st->cfg.max_new) return GREST_EINVAL;
  if (st->variant == GREST_RSVD && n_new > 0 && !omega) return GREST_EINVAL;
  if (where != GREST_HOST && where != GREST_DEVICE) return GREST_EINVAL;
  if (where == GREST_HOST && !host_changes_ok(st->n, n_new, n_changes, ei, ej, sign)) return GREST_EINVAL;
  // the previous update may still run on the device: its status (and stage times) are
  // collected at this update's validation wait
  grest_status rc = st->es == 8 ? update_impl<double>(st, n_new, n_changes, ei, ej, sign, omega, where)
                                : update_impl<float>(st, n_new, n_changes, ei, ej, sign, omega, where);
  if (st->batch) {  // a batch member: its stages are all queued, the others need not wait for it
    batch_leave(st->batch);
    st->batch = nullptr;
  }
  if (rc != GREST_OK || st->rs_every <= 0) return rc;
  // restart policy: the drift is measured once every rs_every updates (this call then
  // waits for the update); past a threshold the pairs are recomputed from scratch, at
  // most once every rs_gap updates
  ++st->rs_since_check;
  ++st->rs_since_start;
  if (st->rs_since_check < st->rs_every) return GREST_OK;
  st->rs_since_check = 0;
  double o = 0.0, r = 0.0;
  CHK(st->es == 8 ? drift_impl<double>(st, &o, &r) : drift_impl<float>(st, &o, &r));
  st->rs_last_orth = o;
  st->rs_last_resid = r;
  if ((r > st->rs_tol_resid || o > st->rs_tol_orth) && st->rs_since_start >= st->rs_gap) {
    // keep the update's numerical status for grest_sync: the restart reuses the word
    st->deferred |= st->pin->status & ST_NUMERIC;
    st->pin->status = 0;
    const uint64_t seed = st->rs_seed + (uint64_t)st->rs_count;
    ++st->rs_count;
    const double tol = default_init_tol(st);
    return st->es == 8 ? init_impl<double>(st, st->rs_iters, tol, seed, nullptr, nullptr)
                       : init_impl<float>(st, st->rs_iters, tol, seed, nullptr, nullptr);
  }
  return GREST_OK;
}

// The change-list buffers of grest_update_noalloc carved out of the static device
// workspace (fixed layout for kNoAllocMaxChanges changes, 256-byte aligned pieces).
// False if the layout does not fit.
bool noalloc_bufs(void* base, ChangeBufs* b) {
  const int64_t nc = kNoAllocMaxChanges;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = (char*)base + off;
    off += (bytes + 255) & ~size_t(255);
    return (void*)p;
  };
  b->ei = (int32_t*)take(nc * sizeof(int32_t));
  b->ej = (int32_t*)take(nc * sizeof(int32_t));
  b->sg = (int8_t*)take(nc);
  b->kin = (uint64_t*)take(2 * nc * sizeof(uint64_t));
  b->kout = (uint64_t*)take(2 * nc * sizeof(uint64_t));
  for (int k = 0; k < 2; ++k) {
    b->dcol[k] = (int32_t*)take(2 * nc * sizeof(int32_t));
    b->dsg[k] = (int8_t*)take(2 * nc);
  }
  b->dins = (int32_t*)take(2 * nc * sizeof(int32_t));
  b->sg_tmp = (int8_t*)take(2 * nc);
  return off <= kNoAllocScratchBytes;
}

grest_status grest_update_noalloc(grest_state* st, int64_t n_new, int64_t n_changes, const int32_t* ei,
                                  const int32_t* ej, const int8_t* sign, const double* omega, int32_t where) {
  if (!st || !st->has_pairs) return GREST_EINVAL;
  if (n_new < 0 || n_changes < 0) return GREST_EINVAL;
  if (st->n + n_new >= INT32_MAX) return GREST_EINVAL;
  if (n_changes > 0 && (!ei || !ej || !sign)) return GREST_EINVAL;
  if (st->variant == GREST_G3 && n_new > st->cfg.max_new) return GREST_EINVAL;
  if (st->variant == GREST_RSVD && n_new > 0 && !omega) return GREST_EINVAL;
  if (where != GREST_HOST && where != GREST_DEVICE) return GREST_EINVAL;
  // nothing may grow: every size the update needs must fit what is already allocated
  auto refuse = [](const char* what) {
    snprintf(g_last_error, sizeof(g_last_error), "grest_update_noalloc: %s", what);
    return GREST_EINVAL;
  };
  const int64_t n2 = st->n + n_new;
  if (n_changes > kNoAllocMaxChanges) return refuse("change list longer than the workspace's maximum");
  if (n2 > st->cap_n) return refuse("node count beyond the state's node capacity");
  if (!st->graph_free && st->m + 2 * n_changes > st->cap_m)
    return refuse("stored entries beyond the state's entry capacity");
  if (st->variant == GREST_RSVD && n_new > st->cap_s)
    return refuse("appended nodes beyond the state's sketch capacity");
  if (st->proj == GREST_PROJ_LOWRANK &&
      std::min<int64_t>(n2, 2 * n_changes) > std::max<int64_t>(1, std::min<int64_t>(2 * st->cap_nc, st->cap_n)))
    return refuse("rows of Delta beyond the low-rank gather capacity");
  // the format of the change list is checked on the device alone (the host check sorts a
  // copy of the keys, which would allocate); a violation still leaves the state unchanged
  void* base = nullptr;
  const hipError_t e = noalloc_scratch(st->device, &base);
  if (e != hipSuccess) {
    set_err("hipGetSymbolAddress of the no-allocation workspace", e);
    return GREST_EDEVICE;
  }
  ChangeBufs cb;
  if (!noalloc_bufs(base, &cb)) return refuse("workspace layout does not fit");
  return st->es == 8 ? update_impl<double>(st, n_new, n_changes, ei, ej, sign, omega, where, &cb)
                     : update_impl<float>(st, n_new, n_changes, ei, ej, sign, omega, where, &cb);
}

grest_status grest_drift(grest_state* st, double* orth, double* resid) {
  if (!st || !st->has_pairs) return GREST_EINVAL;
  return st->es == 8 ? drift_impl<double>(st, orth, resid) : drift_impl<float>(st, orth, resid);
}

grest_status grest_set_restart(grest_state* st, double tol_resid, double tol_orth, int32_t check_every,
                               int32_t min_gap, int32_t iterations, uint64_t seed) {
  if (!st || check_every < 0 || min_gap < 0) return GREST_EINVAL;
  if (check_every > 0 && (iterations < 1 || st->graph_free || !(tol_resid >= 0.0) || !(tol_orth >= 0.0)))
    return GREST_EINVAL;
  st->rs_every = check_every;
  st->rs_gap = min_gap;
  st->rs_iters = iterations;
  st->rs_tol_resid = tol_resid;
  st->rs_tol_orth = tol_orth;
  st->rs_seed = seed;
  st->rs_since_check = 0;
  return GREST_OK;
}

grest_status grest_restart_stats(const grest_state* st, int64_t* restarts, double* last_orth, double* last_resid) {
  if (!st) return GREST_EINVAL;
  if (restarts) *restarts = st->rs_count;
  if (last_orth) *last_orth = st->rs_last_orth;
  if (last_resid) *last_resid = st->rs_last_resid;
  return GREST_OK;
}

grest_status grest_sync(grest_state* st) {
  if (!st) return GREST_EINVAL;
  CHK(sync_all(st));
  prof_collect(st);
  int32_t bits = st->deferred | (st->pin->status & ST_NUMERIC);
  st->deferred = 0;
  st->pin->status = 0;
  if (bits) {
    snprintf(g_last_error, sizeof(g_last_error), "numerical status bits 0x%x", bits);
    return GREST_ENUMERIC;
  }
  return GREST_OK;
}

grest_status grest_get(grest_state* st, double* values, void* X, int32_t x_dtype, int32_t where) {
  if (!st) return GREST_EINVAL;
  if (x_dtype != GREST_F64 && x_dtype != GREST_F32) return GREST_EINVAL;
  if (where != GREST_HOST && where != GREST_DEVICE) return GREST_EINVAL;
  return st->es == 8 ? get_impl<double>(st, values, X, x_dtype, where) : get_impl<float>(st, values, X, x_dtype, where);
}

grest_status grest_shape(const grest_state* st, int64_t* n, int64_t* nnz, int32_t* k, int32_t* width) {
  if (!st) return GREST_EINVAL;
  if (n) *n = st->n;
  if (nnz) *nnz = st->m;
  if (k) *k = st->K;
  if (width) *width = st->D;
  return GREST_OK;
}

grest_status grest_get_graph(grest_state* st, int64_t* rowptr, int32_t* col) {
  if (!st || st->graph_free) return GREST_EINVAL;
  CHK(sync_all(st));
  if (rowptr) HIPCHK(hipMemcpy(rowptr, st->rp[st->gcur], (st->n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
  if (col && st->m > 0) HIPCHK(hipMemcpy(col, st->col[st->gcur], st->m * sizeof(int32_t), hipMemcpyDeviceToHost));
  return GREST_OK;
}

grest_status grest_set_stream(grest_state* st, void* stream) {
  if (!st) return GREST_EINVAL;
  CHK(sync_all(st));
  if (stream) {
    if (st->own_stream) (void)hipStreamDestroy(st->stream);
    st->own_stream = false;
    st->stream = (hipStream_t)stream;
  } else if (!st->own_stream) {
    hipStream_t s = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    st->stream = s;
    st->own_stream = true;
  }
  if (!st->overlap) st->gstream = st->stream;
  return GREST_OK;
}

grest_status grest_set_overlap(grest_state* st, int32_t enable) {
  if (!st) return GREST_EINVAL;
  CHK(sync_all(st));
  if (enable && !st->overlap) {
    hipStream_t g = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&g, hipStreamNonBlocking));
    st->gstream = g;
    st->overlap = true;
  } else if (!enable && st->overlap) {
    (void)hipStreamDestroy(st->gstream);
    st->gstream = st->stream;
    st->overlap = false;
  }
  return GREST_OK;
}

grest_status grest_release_graph(grest_state* st) {
  if (!st) return GREST_EINVAL;
  if (st->proj != GREST_PROJ_LOWRANK) {
    snprintf(g_last_error, sizeof(g_last_error), "only a state with the low-rank projection can drop its graph");
    return GREST_EINVAL;
  }
  if (st->graph_free) return GREST_OK;
  if (st->op != GREST_OP_ADJ) {
    snprintf(g_last_error, sizeof(g_last_error), "a Laplacian state keeps its graph: the shift 2 d_max comes from it");
    return GREST_EINVAL;
  }
  if (st->rs_every > 0) {
    snprintf(g_last_error, sizeof(g_last_error), "a state with a restart policy needs its graph");
    return GREST_EINVAL;
  }
  CHK(sync_all(st));
  // the two CSR column buffers and the product buffer (op Z); the row offsets and the
  // scales are node-sized and stay (unused)
  dfree(st->col[0]);
  dfree(st->col[1]);
  dfree(st->aux);
  st->cap_m = 0;
  st->m = -1;
  st->graph_free = true;
  return GREST_OK;
}

grest_status grest_memory(const grest_state* st, int64_t* bytes) {
  if (!st || !bytes) return GREST_EINVAL;
  *bytes = device_bytes(st);
  return GREST_OK;
}

grest_status grest_profile(grest_state* st, int32_t enable) {
  if (!st) return GREST_EINVAL;
  CHK(sync_all(st));
  if (enable && !st->pev[0][0]) {
    for (int b = 0; b < 2; ++b) {
      for (int i = 0; i <= grest_state::NSTAGE; ++i) HIPCHK(hipEventCreate(&st->pev[b][i]));
      HIPCHK(hipEventCreate(&st->gend[b]));
      HIPCHK(hipEventCreate(&st->kev[b][0]));
      HIPCHK(hipEventCreate(&st->kev[b][1]));
    }
  }
  if (enable < 0 || enable > 2) return GREST_EINVAL;
  st->prof = enable != 0;
  st->stage_marks = enable == 1;
  st->prof_pending[0] = st->prof_pending[1] = false;
  for (int i = 0; i < grest_state::NSTAGE; ++i) st->stage_ms[i] = 0.0;
  st->spmm_ms = 0.0;
  st->prof_spmm_cols = 0;
  st->prof_updates = 0;
  return GREST_OK;
}

grest_status grest_stage_times(grest_state* st, double* stage_ms, int32_t n_stages, double* spmm_ms,
                               int64_t* updates, int64_t* spmm_cols) {
  if (!st) return GREST_EINVAL;
  CHK(sync_all(st));
  prof_collect(st);
  if (stage_ms)
    for (int i = 0; i < n_stages && i < grest_state::NSTAGE; ++i) stage_ms[i] = st->stage_ms[i];
  if (spmm_ms) *spmm_ms = st->spmm_ms;
  if (updates) *updates = st->prof_updates;
  if (spmm_cols) *spmm_cols = st->prof_spmm_cols;
  return GREST_OK;
}

// ---------------------------------------------------------------------------------
// checkpoint / resume and the borrowed view of the tracked block
// ---------------------------------------------------------------------------------
namespace {
struct CheckpointHeader {
  char magic[8];
  int32_t abi, es;
  grest_config cfg;
  int64_t n, m, cap_n, cap_m;
  int32_t has_pairs, graph_free, ax_valid, ax_age;
};
constexpr char kCheckpointMagic[8] = {'G', 'R', 'E', 'S', 'T', 'C', 'K', '1'};

// layout after the header: rowptr (n + 1 int64) and col (m int32) unless the graph was
// released; values (K f64) and X (n x K f64, row-major) with pairs; the kept product
// A X (n x K of the state's element type) when valid
size_t checkpoint_bytes(const CheckpointHeader& h) {
  size_t b = sizeof(CheckpointHeader);
  if (!h.graph_free) b += (size_t)(h.n + 1) * sizeof(int64_t) + (size_t)h.m * sizeof(int32_t);
  if (h.has_pairs) b += (size_t)h.cfg.k * sizeof(double) + (size_t)h.n * h.cfg.k * sizeof(double);
  if (h.ax_valid) b += (size_t)h.n * h.cfg.k * h.es;
  return b;
}
}  // namespace

grest_status grest_save(grest_state* st, void* buf, size_t* bytes) {
  if (!st || !bytes) return GREST_EINVAL;
  CHK(sync_all(st));
  CheckpointHeader h;
  memset(&h, 0, sizeof(h));
  memcpy(h.magic, kCheckpointMagic, sizeof(h.magic));
  h.abi = grest_abi_version();
  h.es = st->es;
  h.cfg = st->cfg;
  h.n = st->n;
  h.m = st->graph_free ? 0 : st->m;
  h.cap_n = st->cap_n;
  h.cap_m = st->cap_m;
  h.has_pairs = st->has_pairs ? 1 : 0;
  h.graph_free = st->graph_free ? 1 : 0;
  h.ax_valid = (st->ax_valid && st->has_pairs && !st->graph_free && st->op == GREST_OP_ADJ &&
                st->proj == GREST_PROJ_EXACT) ? 1 : 0;
  h.ax_age = st->ax_age;
  const size_t need = checkpoint_bytes(h);
  if (!buf || *bytes < need) {
    const bool query = !buf;
    *bytes = need;
    return query ? GREST_OK : GREST_EINVAL;
  }
  char* p = (char*)buf;
  memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  if (!h.graph_free) {
    HIPCHK(hipMemcpy(p, st->rp[st->gcur], (h.n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    p += (h.n + 1) * sizeof(int64_t);
    if (h.m > 0) HIPCHK(hipMemcpy(p, st->col[st->gcur], h.m * sizeof(int32_t), hipMemcpyDeviceToHost));
    p += h.m * sizeof(int32_t);
  }
  if (h.has_pairs) {
    double* vals = (double*)p;
    double* X = vals + h.cfg.k;
    CHK(grest_get(st, vals, X, GREST_F64, GREST_HOST));
    p += (size_t)h.cfg.k * sizeof(double) + (size_t)h.n * h.cfg.k * sizeof(double);
  }
  if (h.ax_valid) {
    HIPCHK(hipMemcpy2D(p, (size_t)h.cfg.k * h.es, st->aux, (size_t)st->ldq * h.es, (size_t)h.cfg.k * h.es, h.n,
                       hipMemcpyDeviceToHost));
  }
  *bytes = need;
  return GREST_OK;
}

grest_status grest_load(const void* buf, size_t bytes, void* stream, grest_state** out) {
  if (!out) return GREST_EINVAL;
  *out = nullptr;
  if (!buf || bytes < sizeof(CheckpointHeader)) return GREST_EINVAL;
  CheckpointHeader h;
  memcpy(&h, buf, sizeof(h));
  if (memcmp(h.magic, kCheckpointMagic, sizeof(h.magic)) != 0 || h.abi != grest_abi_version()) return GREST_EINVAL;
  // everything the sizes and the device copies below depend on is checked before use
  if (h.es != (h.cfg.precision == GREST_FP64 ? 8 : 4)) return GREST_EINVAL;
  if (h.n < 1 || h.n >= INT32_MAX || h.m < 0 || h.m > ((int64_t)1 << 40) || h.cfg.k < 1 || h.cfg.k > 128)
    return GREST_EINVAL;
  if ((h.has_pairs | h.graph_free | h.ax_valid) & ~1) return GREST_EINVAL;
  if (h.graph_free && (h.m != 0 || h.cfg.proj != GREST_PROJ_LOWRANK)) return GREST_EINVAL;
  // the kept product exists only for the exact adjacency form with pairs and a graph
  if (h.ax_valid && (!h.has_pairs || h.graph_free || h.cfg.op != GREST_OP_ADJ || h.cfg.proj != GREST_PROJ_EXACT))
    return GREST_EINVAL;
  if (checkpoint_bytes(h) != bytes) return GREST_EINVAL;
  const char* p = (const char*)buf + sizeof(h);
  std::vector<int64_t> empty_rp;
  const int64_t* rp = nullptr;
  const int32_t* col = nullptr;
  if (h.graph_free) {  // the released graph is not stored: an empty one of n nodes stands in
    empty_rp.assign((size_t)h.n + 1, 0);
    rp = empty_rp.data();
  } else {
    rp = (const int64_t*)p;
    p += (h.n + 1) * sizeof(int64_t);
    col = (const int32_t*)p;
    p += h.m * sizeof(int32_t);
    if (rp[h.n] != h.m) return GREST_EINVAL;
  }
  grest_state* st = nullptr;
  CHK(create_impl(&h.cfg, stream, h.n, rp, col, h.cap_n, h.graph_free ? 1 : h.cap_m, true, &st));
  grest_status rc = GREST_OK;
  if (h.graph_free) rc = grest_release_graph(st);
  if (rc == GREST_OK && h.has_pairs) {
    const double* vals = (const double*)p;
    const double* X = vals + h.cfg.k;
    rc = grest_set_pairs(st, vals, X, GREST_HOST);
    p += (size_t)h.cfg.k * sizeof(double) + (size_t)h.n * h.cfg.k * sizeof(double);
  }
  if (rc == GREST_OK && h.ax_valid) {
    if (hipMemcpy2D(st->aux, (size_t)st->ldq * h.es, p, (size_t)h.cfg.k * h.es, (size_t)h.cfg.k * h.es, h.n,
                    hipMemcpyHostToDevice) != hipSuccess) {
      rc = GREST_EDEVICE;
    } else {
      st->ax_valid = true;
      st->ax_age = h.ax_age;
    }
  }
  if (rc != GREST_OK) {
    grest_destroy(st);
    return rc;
  }
  *out = st;
  return GREST_OK;
}

grest_status grest_view(grest_state* st, const void** X, int64_t* n, int64_t* ld, int32_t* dtype) {
  if (!st || !st->has_pairs) return GREST_EINVAL;
  if (X) *X = st->z[st->zcur];
  if (n) *n = st->n;
  if (ld) *ld = st->ldz;
  if (dtype) *dtype = st->es == 8 ? GREST_F64 : GREST_F32;
  return GREST_OK;
}

void grest_destroy(grest_state* st) {
  if (!st) return;
  (void)sync_all(st);
  if (st->overlap) (void)hipStreamDestroy(st->gstream);
  for (int b = 0; b < 2; ++b) {
    if (st->gend[b]) (void)hipEventDestroy(st->gend[b]);
    for (int i = 0; i <= grest_state::NSTAGE; ++i)
      if (st->pev[b][i]) (void)hipEventDestroy(st->pev[b][i]);
    if (st->kev[b][0]) (void)hipEventDestroy(st->kev[b][0]);
    if (st->kev[b][1]) (void)hipEventDestroy(st->kev[b][1]);
  }
  free_all(st);
  if (st->own_stream) (void)hipStreamDestroy(st->stream);
  delete st;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// Batched updates of many graphs (lockstep one-workgroup stages)
// ---------------------------------------------------------------------------------
namespace {

// Helper threads for the members of a batch beyond the caller's own, kept for reuse.
struct BatchRunner {
  BatchCtx* bc = nullptr;
  int device = 0;
  int size = 0;  // members it can run
  std::vector<std::thread> helpers;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  uint64_t gen = 0;
  int count = 0, remaining = 0;
  bool stop = false;
  const std::function<void(int)>* task = nullptr;

  void helper(int idx) {
    (void)hipSetDevice(device);
    uint64_t seen = 0;
    for (;;) {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || gen != seen; });
      if (stop) return;
      seen = gen;
      if (idx >= count) continue;
      const std::function<void(int)>* f = task;
      lk.unlock();
      (*f)(idx);
      lk.lock();
      if (--remaining == 0) cv_done.notify_all();
    }
  }
  // runs f(0) on the calling thread and f(1 .. count - 1) on the helpers, then returns
  void run(int n, const std::function<void(int)>& f) {
    {
      std::lock_guard<std::mutex> lk(mu);
      task = &f;
      count = n;
      remaining = n - 1;
      ++gen;
    }
    cv.notify_all();
    f(0);
    std::unique_lock<std::mutex> lk(mu);
    cv_done.wait(lk, [&] { return remaining == 0; });
  }
  ~BatchRunner() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    for (auto& t : helpers) t.join();
    batch_destroy(bc);
  }
};

std::mutex g_runner_mu;
std::vector<BatchRunner*> g_runners_free;  // idle runners (any device, any size)

BatchRunner* runner_take(int device, int size) {
  {
    std::lock_guard<std::mutex> lk(g_runner_mu);
    for (size_t i = 0; i < g_runners_free.size(); ++i)
      if (g_runners_free[i]->device == device && g_runners_free[i]->size >= size) {
        BatchRunner* r = g_runners_free[i];
        g_runners_free.erase(g_runners_free.begin() + i);
        return r;
      }
  }
  BatchRunner* r = new BatchRunner;
  r->device = device;
  r->size = std::max(size, 8);
  r->bc = batch_create(device, r->size);
  if (!r->bc) {
    delete r;
    return nullptr;
  }
  for (int i = 1; i < r->size; ++i) r->helpers.emplace_back(&BatchRunner::helper, r, i);
  return r;
}

void runner_give(BatchRunner* r) {
  std::lock_guard<std::mutex> lk(g_runner_mu);
  g_runners_free.push_back(r);
}

}  // namespace

grest_status grest_update_batch(grest_batch_item* items, int32_t count) {
  if (!items || count < 1 || count > GREST_BATCH_MAX) return GREST_EINVAL;
  for (int i = 0; i < count; ++i) {
    items[i].status = GREST_EINVAL;
    if (!items[i].state) return GREST_EINVAL;
    for (int j = 0; j < i; ++j)
      if (items[j].state == items[i].state) return GREST_EINVAL;
    if (items[i].state->device != items[0].state->device || items[i].state->batch) return GREST_EINVAL;
  }
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  const int device = items[0].state->device;
  if (cur != device) HIPCHK(hipSetDevice(device));
  BatchRunner* r = runner_take(device, count);
  if (!r) {
    for (int i = 0; i < count; ++i) items[i].status = GREST_ENOMEM;
    if (cur != device) (void)hipSetDevice(cur);
    snprintf(g_last_error, sizeof(g_last_error), "could not set up a batch of %d", count);
    return GREST_ENOMEM;
  }
  batch_begin(r->bc, count);
  std::vector<std::string> errs(count);
  const std::function<void(int)> member = [&](int i) {
    grest_batch_item& it = items[i];
    grest_state* st = it.state;
    st->batch = r->bc;
    st->batch_err = 0;
    grest_status rc = grest_update(st, it.n_new, it.n_changes, it.ei, it.ej, it.sign, it.omega, it.where);
    if (st->batch) {  // returned before its update was queued
      batch_leave(st->batch);
      st->batch = nullptr;
    }
    if (rc == GREST_OK && st->batch_err) rc = (grest_status)st->batch_err;
    if (rc != GREST_OK) errs[i] = g_last_error;
    it.status = rc;
  };
  r->run(count, member);
  runner_give(r);
  if (cur != device) (void)hipSetDevice(cur);
  for (int i = 0; i < count; ++i)
    if (items[i].status != GREST_OK) {
      snprintf(g_last_error, sizeof(g_last_error), "batch member %d: %s", i, errs[i].c_str());
      return (grest_status)items[i].status;
    }
  return GREST_OK;
}
