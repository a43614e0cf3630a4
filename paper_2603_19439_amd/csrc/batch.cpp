// Lockstep execution of the one-workgroup stages of many graphs' updates.
//
// Every member of a batch runs its own graph's update on its own host thread and its own
// stream.  At a one-workgroup stage (a CholQR factor, a small eigensolve) a member does not
// launch: it records an event on its stream, hands over its job descriptor and waits.  When
// every member still running has arrived, the last one to arrive launches the stage for all
// of them at once on the batch stream: that stream waits for the members' events, the jobs
// go to device memory as one descriptor array, the batched kernels run one workgroup per
// graph (per graph and pair for the eigenvector kernels), and every member's stream then
// waits for the batch stream's event.  Members at different stages in the same round are
// served by the same round (each stage has its own launches).  A member whose update has no
// stage left leaves, so the others never wait for it.
//
// Nothing is reordered on the device but the one-workgroup kernels, which run with exactly
// the arguments of their single-graph launch: the members' results are those of the same
// updates run one at a time.
//
// The launches of a round depend only on its shape: which kernel instances, how many jobs
// each, and the block counts of the per-pair kernels.  The first round of a shape is
// captured from the batch stream into a HIP graph whose kernels read a descriptor array of
// their own; a later round of the same shape copies its descriptors there and replays the
// graph, one launch instead of up to ten (GREST_BATCH_GRAPHS=0 in the environment launches
// every round directly instead).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/grest.h"
#include "grest_internal.h"

namespace {

constexpr size_t kRingBytes = 1 << 20;  // descriptor staging, reused once the stream has drained
constexpr size_t kMaxGraphs = 256;       // captured round shapes kept per batch context

// A captured round: its graph and the descriptor arrays its kernels read.
struct RoundGraph {
  hipGraphExec_t exec = nullptr;
  void* chol = nullptr;  // device arrays, as many jobs as the shape has
  void* eig = nullptr;
};

struct Pending {
  int kind;  // 0: factor, 1: eigensolve
  CholJob chol;
  EigJob eig;
  hipStream_t stream;
  int slot;  // event slot
};

}  // namespace

struct BatchCtx {
  int device = 0;
  int max_members = 0;
  int members = 0;  // still running
  uint64_t gen = 0;
  int error = 0;  // first failed device call of a round
  std::mutex mu;
  std::condition_variable cv;
  std::vector<Pending> pend;
  std::vector<hipEvent_t> ev;  // one per arrival slot of a round
  hipEvent_t done = nullptr;
  hipStream_t bs = nullptr;
  unsigned char* host_ring = nullptr;  // pinned
  unsigned char* dev_ring = nullptr;
  size_t ring_off = 0;
  bool graphs = true;
  std::map<std::vector<int>, RoundGraph> cache;  // by round shape
};

namespace {

int hip_fail(hipError_t e) { return e == hipSuccess ? 0 : (int)GREST_EDEVICE; }

// staging space for `bytes` of descriptors: the host part is rewritten only after the
// batch stream has finished reading what an earlier round put there
int ring_take(BatchCtx* bc, size_t bytes, size_t* off) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (bytes > kRingBytes) return GREST_EINVAL;
  if (bc->ring_off + bytes > kRingBytes) {
    if (int rc = hip_fail(hipStreamSynchronize(bc->bs))) return rc;
    bc->ring_off = 0;
  }
  *off = bc->ring_off;
  bc->ring_off += bytes;
  return 0;
}

template <typename J>
int stage_jobs(BatchCtx* bc, std::vector<J>& jobs, J** dev) {
  size_t off = 0;
  const size_t bytes = jobs.size() * sizeof(J);
  if (int rc = ring_take(bc, bytes, &off)) return rc;
  std::memcpy(bc->host_ring + off, jobs.data(), bytes);
  *dev = reinterpret_cast<J*>(bc->dev_ring + off);
  return hip_fail(hipMemcpyAsync(*dev, bc->host_ring + off, bytes, hipMemcpyHostToDevice, bc->bs));
}

// shape of a round: per job its kernel instance, its block counts and the sizes its dynamic
// LDS depends on, in launch order
std::vector<int> round_shape(const std::vector<CholJob>& cj, const std::vector<EigJob>& ej) {
  std::vector<int> k;
  k.push_back((int)cj.size());
  for (const CholJob& j : cj) {  // the instance, and the order and coefficient rows that size its LDS
    k.push_back(chol_job_key(j));
    k.push_back(j.m);
    k.push_back(j.C ? j.kc : 0);
  }
  k.push_back((int)ej.size());
  for (const EigJob& j : ej) {
    k.push_back(eig_job_key(j));
    k.push_back(j.d_full);
    k.push_back(j.kk);
  }
  return k;
}

// staging copy of a round's descriptors into device memory at dst, on the batch stream
template <typename J>
int copy_jobs(BatchCtx* bc, const std::vector<J>& jobs, void* dst) {
  if (jobs.empty()) return 0;
  size_t off = 0;
  const size_t bytes = jobs.size() * sizeof(J);
  if (int rc = ring_take(bc, bytes, &off)) return rc;
  std::memcpy(bc->host_ring + off, jobs.data(), bytes);
  return hip_fail(hipMemcpyAsync(dst, bc->host_ring + off, bytes, hipMemcpyHostToDevice, bc->bs));
}

void launch_sets(std::vector<CholJob>& cj, std::vector<EigJob>& ej, void* dchol, void* deig, hipStream_t s) {
  if (!cj.empty()) chol_batch_launch(cj.data(), (const CholJob*)dchol, (int)cj.size(), s);
  if (!ej.empty()) small_eig_batch_launch(ej.data(), (const EigJob*)deig, (int)ej.size(), s);
}

// the round's launches through its captured graph (captured now if its shape is new)
int replay_round(BatchCtx* bc, std::vector<CholJob>& cj, std::vector<EigJob>& ej) {
  const std::vector<int> key = round_shape(cj, ej);
  auto it = bc->cache.find(key);
  if (it == bc->cache.end()) {
    if (bc->cache.size() >= kMaxGraphs) {  // drop every shape kept so far
      if (int rc = hip_fail(hipStreamSynchronize(bc->bs))) return rc;
      for (auto& kv : bc->cache) {
        (void)hipGraphExecDestroy(kv.second.exec);
        (void)hipFree(kv.second.chol);
        (void)hipFree(kv.second.eig);
      }
      bc->cache.clear();
    }
    RoundGraph g;
    int rc = 0;
    if (!cj.empty()) rc = hip_fail(hipMalloc(&g.chol, cj.size() * sizeof(CholJob)));
    if (!rc && !ej.empty()) rc = hip_fail(hipMalloc(&g.eig, ej.size() * sizeof(EigJob)));
    hipGraph_t graph = nullptr;
    if (!rc) rc = hip_fail(hipStreamBeginCapture(bc->bs, hipStreamCaptureModeRelaxed));
    if (!rc) {
      launch_sets(cj, ej, g.chol, g.eig, bc->bs);
      rc = hip_fail(hipStreamEndCapture(bc->bs, &graph));
    }
    if (!rc) rc = hip_fail(hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) {
      (void)hipFree(g.chol);
      (void)hipFree(g.eig);
      return rc;
    }
    it = bc->cache.emplace(key, g).first;
  }
  if (int rc = copy_jobs(bc, cj, it->second.chol)) return rc;
  if (int rc = copy_jobs(bc, ej, it->second.eig)) return rc;
  return hip_fail(hipGraphLaunch(it->second.exec, bc->bs));
}

// under the lock, by the last member to arrive: one launch set for the whole round
void launch_round(BatchCtx* bc) {
  int rc = 0;
  for (const Pending& p : bc->pend)
    if (!rc) rc = hip_fail(hipStreamWaitEvent(bc->bs, bc->ev[p.slot], 0));
  std::vector<CholJob> cj;
  std::vector<EigJob> ej;
  for (const Pending& p : bc->pend) {
    if (p.kind == 0) cj.push_back(p.chol);
    else ej.push_back(p.eig);
  }
  if (!cj.empty()) chol_batch_prepare(cj.data(), (int)cj.size());
  if (!ej.empty()) small_eig_batch_prepare(ej.data(), (int)ej.size());
  if (!rc && bc->graphs) {
    rc = replay_round(bc, cj, ej);
  } else if (!rc) {
    CholJob* dc = nullptr;
    EigJob* de = nullptr;
    if (!cj.empty()) rc = stage_jobs(bc, cj, &dc);
    if (!rc && !ej.empty()) rc = stage_jobs(bc, ej, &de);
    if (!rc) launch_sets(cj, ej, dc, de, bc->bs);
  }
  if (!rc) rc = hip_fail(hipGetLastError());
  if (!rc) rc = hip_fail(hipEventRecord(bc->done, bc->bs));
  for (const Pending& p : bc->pend)
    if (!rc) rc = hip_fail(hipStreamWaitEvent(p.stream, bc->done, 0));
  if (rc && !bc->error) bc->error = rc;
  bc->pend.clear();
  ++bc->gen;
  bc->cv.notify_all();
}

int arrive(BatchCtx* bc, Pending p) {
  std::unique_lock<std::mutex> lk(bc->mu);
  if (bc->error) return bc->error;
  p.slot = (int)bc->pend.size();
  if (int rc = hip_fail(hipEventRecord(bc->ev[p.slot], p.stream))) return rc;
  bc->pend.push_back(p);
  const uint64_t g = bc->gen;
  if ((int)bc->pend.size() >= bc->members) launch_round(bc);
  else bc->cv.wait(lk, [&] { return bc->gen != g; });
  return bc->error;
}

}  // namespace

BatchCtx* batch_create(int device, int max_members) {
  if (max_members < 1) return nullptr;
  BatchCtx* bc = new BatchCtx;
  bc->device = device;
  bc->max_members = max_members;
  bc->ev.resize(max_members, nullptr);
  bool ok = hipStreamCreateWithFlags(&bc->bs, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&bc->done, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; ok && i < max_members; ++i)
    ok = hipEventCreateWithFlags(&bc->ev[i], hipEventDisableTiming) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&bc->host_ring, kRingBytes, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipMalloc((void**)&bc->dev_ring, kRingBytes) == hipSuccess;
  const char* env = std::getenv("GREST_BATCH_GRAPHS");
  bc->graphs = !(env && env[0] == '0');
  batch_kernels_init();  // kernel attributes, before any capture
  if (!ok) {
    batch_destroy(bc);
    return nullptr;
  }
  return bc;
}

void batch_destroy(BatchCtx* bc) {
  if (!bc) return;
  if (bc->bs) (void)hipStreamSynchronize(bc->bs);
  for (auto& kv : bc->cache) {
    (void)hipGraphExecDestroy(kv.second.exec);
    (void)hipFree(kv.second.chol);
    (void)hipFree(kv.second.eig);
  }
  for (hipEvent_t e : bc->ev)
    if (e) (void)hipEventDestroy(e);
  if (bc->done) (void)hipEventDestroy(bc->done);
  if (bc->host_ring) (void)hipHostFree(bc->host_ring);
  if (bc->dev_ring) (void)hipFree(bc->dev_ring);
  if (bc->bs) (void)hipStreamDestroy(bc->bs);
  delete bc;
}

void batch_begin(BatchCtx* bc, int members) {
  std::lock_guard<std::mutex> lk(bc->mu);
  bc->members = std::min(members, bc->max_members);
  bc->error = 0;
  bc->pend.clear();
}

int batch_chol(BatchCtx* bc, hipStream_t s, const CholJob& job) {
  Pending p{};
  p.kind = 0;
  p.chol = job;
  p.stream = s;
  return arrive(bc, p);
}

int batch_small_eig(BatchCtx* bc, hipStream_t s, const EigJob& job) {
  Pending p{};
  p.kind = 1;
  p.eig = job;
  p.stream = s;
  return arrive(bc, p);
}

void batch_leave(BatchCtx* bc) {
  std::lock_guard<std::mutex> lk(bc->mu);
  --bc->members;
  if (bc->members > 0 && (int)bc->pend.size() >= bc->members) launch_round(bc);
}
