// Continuous-batching request loop for eigen-solves on one GPU.
//
// Requests are admitted while the sum of their device footprints fits the
// context budget (a request alone is always admitted once nothing runs).  A
// fixed pool of workers runs the admitted requests, each on a stream and a
// workspace of its own, so the inner iterations of all resident requests are
// in flight on the device together and a request arriving while others run
// starts as soon as a worker and memory free up.  A worker keeps its
// workspace for the next queued request of the same shape.  No arithmetic is
// shared between requests, so a result does not depend on its neighbours.
#pragma once

#include "engine.h"

namespace ifeast {

struct Request;

struct Server {
  explicit Server(ifeast_ctx* ctx);
  // Requests still queued fail with IFEAST_ERR_DEVICE; running ones finish first.  Threads
  // blocked in wait() are released before the server goes away.
  ~Server();
  uint64_t submit(const ifeast_csr* A, const ifeast_csr* B, const ifeast_contour& C, const ifeast_params& p,
                  const double* X0, uint64_t footprint);
  int poll(uint64_t ticket, int* done);
  // Blocks until the request is done; returns its status (an error's text is left in the
  // context's last error before the call returns, so a concurrent destroy never races it).
  int wait(uint64_t ticket, ifeast_result* res, double* latency_s);

  static constexpr int kWorkers = 8;  // requests in flight on the device at once

 private:
  void worker_loop();
  void run(Request* r, ifeast_ctx* sub);
  bool admissible() const;

  ifeast_ctx* ctx_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Request*> queue_;
  std::map<uint64_t, std::unique_ptr<Request>> all_;
  std::vector<std::thread> workers_;
  uint64_t next_ = 1, used_ = 0;
  int running_ = 0;
  int waiters_ = 0;  // threads inside wait()
  bool stop_ = false;
};

// Drop the engine (workspace) a context keeps for its last solve shape.
void release_engine(ifeast_ctx* ctx);

}  // namespace ifeast
