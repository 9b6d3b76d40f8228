// Per-kernel-class event timing (see KernelTimer in internal.h).
#include "internal.h"

namespace ifeast {

KernelTimer*& current_timer() {
  thread_local KernelTimer* t = nullptr;
  return t;
}

KernelTimer::~KernelTimer() {
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

int KernelTimer::begin(hipStream_t st) {
  constexpr int kPool = 512;  // 256 launches between flushes
  if (pool.empty()) {
    pool.resize(kPool);
    for (auto& e : pool) IF_HIP(hipEventCreate(&e));
  }
  if (stream != nullptr && stream != st) flush();
  if (next + 2 > (int)pool.size()) flush();
  stream = st;
  const int tok = next;
  next += 2;
  IF_HIP(hipEventRecord(pool[tok], st));
  return tok;
}

void KernelTimer::end(int tok, int cls, double flops, double bytes) {
  IF_HIP(hipEventRecord(pool[tok + 1], stream));
  pend.push_back({tok, cls, flops, bytes});
}

void KernelTimer::flush() {
  if (pend.empty()) {
    next = 0;
    return;
  }
  IF_HIP(hipEventSynchronize(pool[pend.back().ev + 1]));
  for (const Pending& p : pend) {
    float ms = 0.f;
    IF_HIP(hipEventElapsedTime(&ms, pool[p.ev], pool[p.ev + 1]));
    KernelStat& a = acc[p.cls];
    a.launches += 1;
    a.seconds += ms * 1e-3;
    a.flops += p.flops;
    a.bytes += p.bytes;
  }
  pend.clear();
  next = 0;
}

}  // namespace ifeast
