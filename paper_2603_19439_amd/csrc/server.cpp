// Batched execution of many independent graphs on one device (the serving loop).
//
// A server runs `lanes` worker threads, each with its own HIP streams (default priority).
// Requests wait in one queue in submission order.  A free lane takes the oldest request
// whose graph is not being updated by another lane, moves that graph's state onto its
// own stream (the state is idle then, so the move costs no wait) and runs the request as
// a complete single-graph update (grest_update, then grest_sync for the deferred status).
// With batches (max_batch > 1) a free lane takes up to max_batch such requests, of
// distinct graphs, oldest first, puts each graph on one of its max_batch streams and runs
// them as one grest_update_batch: their one-workgroup stages are launched together.
// So one graph's updates stay ordered and never overlap, no lane idles while a runnable
// request waits behind a long update of another graph, and the lanes overlap on the
// device.  Requests own copies of their change lists.  Completions are kept until
// grest_poll hands them out.
//
// Admission by device memory: the server reserves, for every attached graph, its current
// footprint plus the growth its queued requests will cause (the capacities an update
// grows are known on the host: node and entry buffers by 1.5x, change and sketch buffers
// by 2x).  A submission whose growth would take the reservations past the budget is
// refused with GREST_EAGAIN and can be retried once memory frees up: when a graph with
// nothing queued is detached, and when a graph's requests have all run and its
// reservation is replaced by its actual footprint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/grest.h"
#include "grest_internal.h"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  int32_t gid = 0;
  uint64_t tag = 0;
  int64_t n_new = 0;
  std::vector<int32_t> ei, ej;
  std::vector<int8_t> sg;
  std::vector<double> omega;
  bool has_omega = false;
  int64_t t_submit = 0;
};

struct Done {
  uint64_t tag;
  int32_t status;
  int64_t t_submit, t_done;
};

struct Graph {
  grest_state* st;
  void* user_stream;  // restored on detach or destroy (null: the state had its own stream)
  int64_t bytes;      // reserved device bytes: the footprint once its queued requests have run
  int64_t sketch_cols;  // L + P of an RSVD state, else 0
  StateCaps proj;       // capacities and sizes once every queued request of the graph has run
  int32_t slot;         // server stream the state is on (lane * max_batch + member)
  int32_t k;            // tracked pairs
  int32_t queued;       // its requests queued or running
  bool running;         // a lane is updating it
  bool detached;
};

}  // namespace

struct grest_server {
  int device = 0;
  int64_t budget = 0, used = 0;
  int32_t nlanes = 0, max_queue = 0, max_batch = 1;
  std::vector<hipStream_t> streams;  // lane l's streams: [l * max_batch, (l + 1) * max_batch)
  std::deque<Request> queue;  // submission order
  std::vector<std::thread> workers;
  std::vector<Graph> graphs;
  std::deque<Done> done;
  std::mutex mu;
  std::condition_variable cv_work, cv_idle;
  int64_t pending = 0;  // queued or running
  bool stop = false;
};

namespace {

// size class of a graph for batching: its K and the octave of its node count
int size_class(const Graph& g) {
  int oct = 0;
  for (int64_t n = std::max<int64_t>(g.proj.n, 1); n > 1; n >>= 1) ++oct;
  return g.k * 64 + oct;
}

// Pinned host staging of one request's change list and test matrix: the update's copies to
// the device then run asynchronously instead of through the runtime's staging of pageable
// memory.  A worker reuses its buffers once the updates that read them have been synced.
struct PinnedStage {
  unsigned char* p = nullptr;
  size_t cap = 0;
  PinnedStage() = default;
  PinnedStage(const PinnedStage&) = delete;
  PinnedStage& operator=(const PinnedStage&) = delete;
  ~PinnedStage() {
    if (p) (void)hipHostFree(p);
  }
  // the request's arrays in pinned memory (null where the request has none); false if the
  // buffer cannot be grown, in which case the caller passes the request's own arrays
  bool stage(const Request& rq, const int32_t** ei, const int32_t** ej, const int8_t** sg, const double** om) {
    const size_t nc = rq.ei.size();
    const size_t o_ej = nc * sizeof(int32_t), o_sg = 2 * o_ej;
    const size_t o_om = (o_sg + nc + 7) & ~(size_t)7;
    const size_t bytes = o_om + (rq.has_omega ? rq.omega.size() * sizeof(double) : 0);
    if (bytes > cap) {
      if (p) (void)hipHostFree(p);
      p = nullptr;
      cap = 0;
      const size_t want = std::max<size_t>(bytes, 2 * bytes);
      if (hipHostMalloc((void**)&p, want) != hipSuccess) { p = nullptr; return false; }
      cap = want;
    }
    if (nc) {
      std::memcpy(p, rq.ei.data(), o_ej);
      std::memcpy(p + o_ej, rq.ej.data(), o_ej);
      std::memcpy(p + o_sg, rq.sg.data(), nc);
    }
    if (rq.has_omega) std::memcpy(p + o_om, rq.omega.data(), rq.omega.size() * sizeof(double));
    *ei = nc ? reinterpret_cast<const int32_t*>(p) : nullptr;
    *ej = nc ? reinterpret_cast<const int32_t*>(p + o_ej) : nullptr;
    *sg = nc ? reinterpret_cast<const int8_t*>(p + o_sg) : nullptr;
    *om = rq.has_omega ? reinterpret_cast<const double*>(p + o_om) : nullptr;
    return true;
  }
};

void worker(grest_server* sv, int lane) {
  (void)hipSetDevice(sv->device);
  const int nb = sv->max_batch;
  std::vector<PinnedStage> pins(nb);
  std::vector<Request> rqs;
  std::vector<grest_state*> sts;
  std::vector<bool> moves;
  std::vector<grest_batch_item> items;
  for (;;) {
    rqs.clear();
    sts.clear();
    moves.clear();
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      // the oldest requests whose graphs are idle (a graph's own requests are in order),
      // at most one per graph
      auto runnable = [&] {
        for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it)
          if (!sv->graphs[it->gid].running) return true;
        return false;
      };
      sv->cv_work.wait(lk, [&] { return runnable() || (sv->stop && sv->queue.empty()); });
      if (!runnable()) return;  // stop requested and nothing left
      // a batch holds graphs of one size class (the oldest runnable request's): members in
      // lockstep wait for each other at every one-workgroup stage
      int cls = -1;
      for (auto it = sv->queue.begin(); it != sv->queue.end() && (int)rqs.size() < nb;) {
        Graph& g = sv->graphs[it->gid];  // under the lock: attach may grow the table
        const int c = size_class(g);
        if (g.running || (cls >= 0 && c != cls)) {
          ++it;
          continue;
        }
        cls = c;
        g.running = true;
        const int32_t slot = lane * nb + (int32_t)rqs.size();
        moves.push_back(g.slot != slot);
        g.slot = slot;
        sts.push_back(g.st);
        rqs.push_back(std::move(*it));
        it = sv->queue.erase(it);
      }
    }
    // each state is idle (its last update ended with grest_sync), while its old stream may
    // be running another graph's update: no wait on that stream
    const int cnt = (int)rqs.size();
    for (int i = 0; i < cnt; ++i)
      if (moves[i]) state_rebind_stream(sts[i], sv->streams[lane * nb + i]);
    std::vector<grest_status> ru(cnt, GREST_OK);
    // each member's arrays, staged in pinned memory (the request's own arrays if staging fails)
    struct Args {
      const int32_t *ei, *ej;
      const int8_t* sg;
      const double* om;
    };
    std::vector<Args> args(cnt);
    for (int i = 0; i < cnt; ++i) {
      const Request& rq = rqs[i];
      Args& a = args[i];
      if (!pins[i].stage(rq, &a.ei, &a.ej, &a.sg, &a.om)) {
        const bool has = !rq.ei.empty();
        a = Args{has ? rq.ei.data() : nullptr, has ? rq.ej.data() : nullptr, has ? rq.sg.data() : nullptr,
                 rq.has_omega ? rq.omega.data() : nullptr};
      }
    }
    if (cnt == 1) {
      const Request& rq = rqs[0];
      const int64_t nc = (int64_t)rq.ei.size();
      ru[0] = grest_update(sts[0], rq.n_new, nc, args[0].ei, args[0].ej, args[0].sg, args[0].om, GREST_HOST);
    } else {
      items.assign(cnt, grest_batch_item{});
      for (int i = 0; i < cnt; ++i) {
        const Request& rq = rqs[i];
        const int64_t nc = (int64_t)rq.ei.size();
        items[i] = grest_batch_item{sts[i], rq.n_new, nc, args[i].ei, args[i].ej, args[i].sg, args[i].om,
                                    GREST_HOST, GREST_OK};
      }
      (void)grest_update_batch(items.data(), cnt);  // every member's own status is in its item
      for (int i = 0; i < cnt; ++i) ru[i] = (grest_status)items[i].status;
    }
    for (int i = 0; i < cnt; ++i) {
      const Request& rq = rqs[i];
      grest_state* st = sts[i];
      // waits for the update and reads its deferred numerical status (the update has
      // committed even when that status is not OK)
      const grest_status rs = grest_sync(st);
      const grest_status rc = ru[i] != GREST_OK ? ru[i] : rs;
      const int64_t t_done = now_ns();
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        Graph& g = sv->graphs[rq.gid];
        g.running = false;
        if (--g.queued == 0) {
          // nothing else queued for the graph: its reservation becomes its actual footprint
          // (a rejected request did not grow it; the capacities may have grown by less)
          int64_t actual = g.bytes;
          if (grest_memory(st, &actual) == GREST_OK) {
            sv->used += actual - g.bytes;
            g.bytes = actual;
          }
          state_caps(st, &g.proj);
        }
        sv->done.push_back(Done{rq.tag, (int32_t)rc, rq.t_submit, t_done});
        --sv->pending;
      }
      sv->cv_idle.notify_all();
      sv->cv_work.notify_all();  // the graph's next request may be runnable now
    }
  }
}

}  // namespace

extern "C" {

int64_t grest_now_ns(void) { return now_ns(); }

grest_status grest_server_create(int64_t hbm_budget_bytes, int32_t lanes, int32_t max_queue, grest_server** out) {
  return grest_server_create_batched(hbm_budget_bytes, lanes, max_queue, 1, out);
}

grest_status grest_server_create_batched(int64_t hbm_budget_bytes, int32_t lanes, int32_t max_queue,
                                         int32_t max_batch, grest_server** out) {
  if (!out) return GREST_EINVAL;
  *out = nullptr;
  if (lanes < 1 || lanes > 64 || max_queue < 1 || hbm_budget_bytes < 0) return GREST_EINVAL;
  if (max_batch < 1 || max_batch > GREST_BATCH_MAX || lanes * max_batch > 256) return GREST_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return GREST_ENODEV;
  grest_server* sv = new (std::nothrow) grest_server();
  if (!sv) return GREST_ENOMEM;
  (void)hipGetDevice(&sv->device);
  sv->budget = hbm_budget_bytes;
  sv->nlanes = lanes;
  sv->max_queue = max_queue;
  sv->max_batch = max_batch;
  for (int l = 0; l < lanes * max_batch; ++l) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t t : sv->streams) (void)hipStreamDestroy(t);
      delete sv;
      return GREST_EDEVICE;
    }
    sv->streams.push_back(s);
  }
  for (int l = 0; l < lanes; ++l) sv->workers.emplace_back(worker, sv, l);
  *out = sv;
  return GREST_OK;
}

grest_status grest_server_attach(grest_server* sv, grest_state* st, int32_t* graph_id) {
  if (!sv || !st || !graph_id) return GREST_EINVAL;
  int64_t bytes = 0;
  grest_status rc = grest_memory(st, &bytes);
  if (rc != GREST_OK) return rc;
  int64_t n = 0;
  int32_t k = 0, width = 0;
  if ((rc = grest_shape(st, &n, nullptr, &k, &width)) != GREST_OK) return rc;
  std::lock_guard<std::mutex> lk(sv->mu);
  for (const Graph& g : sv->graphs)
    if (!g.detached && g.st == st) return GREST_EINVAL;  // already attached
  if (sv->budget > 0 && sv->used + bytes > sv->budget) return GREST_EAGAIN;
  const int32_t id = (int32_t)sv->graphs.size();
  void* user = state_user_stream(st);
  const int32_t slot = (id % sv->nlanes) * sv->max_batch;
  if ((rc = grest_set_stream(st, sv->streams[slot])) != GREST_OK) return rc;
  Graph g{st, user, bytes, state_sketch_cols(st), StateCaps{}, slot, k, 0, false, false};
  state_caps(st, &g.proj);
  sv->graphs.push_back(g);
  sv->used += bytes;
  *graph_id = id;
  return GREST_OK;
}

grest_status grest_submit(grest_server* sv, int32_t graph_id, int64_t n_new, int64_t n_changes, const int32_t* ei,
                          const int32_t* ej, const int8_t* sign, const double* omega, uint64_t tag) {
  if (!sv || n_new < 0 || n_changes < 0) return GREST_EINVAL;
  if (n_changes > 0 && (!ei || !ej || !sign)) return GREST_EINVAL;
  Graph g;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (graph_id < 0 || graph_id >= (int32_t)sv->graphs.size() || sv->graphs[graph_id].detached)
      return GREST_EINVAL;
    g = sv->graphs[graph_id];
  }
  if (g.sketch_cols > 0 && n_new > 0 && !omega) return GREST_EINVAL;
  // format, id ranges, no duplicates: against the size the graph will have when this runs
  // (its requests are submitted from one thread, so the size cannot change meanwhile)
  if (grest_validate_changes(g.proj.n, n_new, n_changes, ei, ej, sign) != GREST_OK) return GREST_EINVAL;
  int64_t dm = 0;  // change of the stored entries: +2 per insertion, -2 per deletion
  for (int64_t c = 0; c < n_changes; ++c) dm += sign[c] > 0 ? 2 : -2;
  Request rq;
  rq.gid = graph_id;
  rq.tag = tag;
  rq.n_new = n_new;
  rq.ei.assign(ei, ei + n_changes);
  rq.ej.assign(ej, ej + n_changes);
  rq.sg.assign(sign, sign + n_changes);
  if (omega && g.sketch_cols > 0 && n_new > 0) {
    rq.omega.assign(omega, omega + (size_t)n_new * (size_t)g.sketch_cols);
    rq.has_omega = true;
  }
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->pending >= sv->max_queue) return GREST_EAGAIN;
    Graph& gr = sv->graphs[graph_id];
    if (gr.detached) return GREST_EINVAL;
    StateCaps after = gr.proj;
    state_caps_after(gr.st, &after, n_new, n_changes, dm);
    const int64_t growth = state_bytes_for(gr.st, after) - state_bytes_for(gr.st, gr.proj);
    if (sv->budget > 0 && growth > 0 && sv->used + growth > sv->budget) return GREST_EAGAIN;
    if (growth > 0) {
      sv->used += growth;
      gr.bytes += growth;
    }
    gr.proj = after;
    ++gr.queued;
    rq.t_submit = now_ns();
    sv->queue.push_back(std::move(rq));
    ++sv->pending;
  }
  sv->cv_work.notify_all();
  return GREST_OK;
}

int32_t grest_poll(grest_server* sv, int32_t max, uint64_t* tags, int32_t* status, int64_t* t_submit_ns,
                   int64_t* t_done_ns) {
  if (!sv || max <= 0) return 0;
  std::lock_guard<std::mutex> lk(sv->mu);
  int32_t c = 0;
  while (c < max && !sv->done.empty()) {
    const Done& d = sv->done.front();
    if (tags) tags[c] = d.tag;
    if (status) status[c] = d.status;
    if (t_submit_ns) t_submit_ns[c] = d.t_submit;
    if (t_done_ns) t_done_ns[c] = d.t_done;
    sv->done.pop_front();
    ++c;
  }
  return c;
}

grest_status grest_server_detach(grest_server* sv, int32_t graph_id) {
  if (!sv) return GREST_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (graph_id < 0 || graph_id >= (int32_t)sv->graphs.size() || sv->graphs[graph_id].detached)
    return GREST_EINVAL;
  Graph& g = sv->graphs[graph_id];
  if (g.queued > 0 || g.running) return GREST_EAGAIN;
  // the state is idle: its last update ended with grest_sync on its lane's stream
  grest_status rc = grest_set_stream(g.st, g.user_stream);
  if (rc != GREST_OK) return rc;
  sv->used -= g.bytes;
  g.bytes = 0;
  g.detached = true;
  g.st = nullptr;
  return GREST_OK;
}

grest_status grest_server_memory(grest_server* sv, int64_t* reserved, int64_t* budget) {
  if (!sv) return GREST_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (reserved) *reserved = sv->used;
  if (budget) *budget = sv->budget;
  return GREST_OK;
}

grest_status grest_server_drain(grest_server* sv) {
  if (!sv) return GREST_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  sv->cv_idle.wait(lk, [&] { return sv->pending == 0; });
  return GREST_OK;
}

void grest_server_destroy(grest_server* sv) {
  if (!sv) return;
  (void)grest_server_drain(sv);
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  for (std::thread& t : sv->workers) t.join();
  for (const Graph& g : sv->graphs)
    if (!g.detached) (void)grest_set_stream(g.st, g.user_stream);
  for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
  delete sv;
}

}  // extern "C"
