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
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/grest.h"
#include "grest_internal.h"

namespace {

constexpr size_t kRingBytes = 1 << 20;  // descriptor staging, reused once the stream has drained

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
  if (!rc && !cj.empty()) {
    chol_batch_prepare(cj.data(), (int)cj.size());
    CholJob* dev = nullptr;
    rc = stage_jobs(bc, cj, &dev);
    if (!rc) chol_batch_launch(cj.data(), dev, (int)cj.size(), bc->bs);
  }
  if (!rc && !ej.empty()) {
    small_eig_batch_prepare(ej.data(), (int)ej.size());
    EigJob* dev = nullptr;
    rc = stage_jobs(bc, ej, &dev);
    if (!rc) small_eig_batch_launch(ej.data(), dev, (int)ej.size(), bc->bs);
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
  if (!ok) {
    batch_destroy(bc);
    return nullptr;
  }
  return bc;
}

void batch_destroy(BatchCtx* bc) {
  if (!bc) return;
  if (bc->bs) (void)hipStreamSynchronize(bc->bs);
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
