// Continuous-batching request loop for eigen-solves on one GPU.
//
// Requests are admitted while the sum of their device footprints fits the
// context budget; each admitted request owns its matrices, workspace and a
// HIP stream for its whole life, so the inner iterations of all resident
// requests are in flight on the device together and a request arriving
// while others run starts as soon as memory frees up.  No arithmetic is
// shared between requests, so a result does not depend on its neighbours.
#pragma once

#include "engine.h"

namespace ifeast {

struct Request;

struct Server {
  explicit Server(ifeast_ctx* ctx);
  ~Server();
  uint64_t submit(const ifeast_csr* A, const ifeast_csr* B, const ifeast_contour& C, const ifeast_params& p,
                  const double* X0, uint64_t footprint);
  int poll(uint64_t ticket, int* done);
  int wait(uint64_t ticket, ifeast_result* res, double* latency_s);

 private:
  void dispatch_loop();
  void run(Request* r);

  ifeast_ctx* ctx_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Request*> queue_;
  std::map<uint64_t, std::unique_ptr<Request>> all_;
  std::vector<std::thread> workers_;
  uint64_t next_ = 1, used_ = 0;
  int running_ = 0;
  bool stop_ = false;
  std::thread dispatcher_;
};

}  // namespace ifeast
