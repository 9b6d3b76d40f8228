#include "serve.h"

#include <chrono>

namespace ifeast {

namespace {
using clock_t_ = std::chrono::steady_clock;
}  // namespace

struct Request {
  uint64_t ticket = 0, footprint = 0;
  int64_t n = 0;
  std::vector<int64_t> rpA, rpB;
  std::vector<int32_t> ciA, ciB;
  std::vector<double> vA, vB, X0, cz, cw;
  bool hasB = false, hasX0 = false;
  ifeast_contour C{};
  ifeast_params p{};
  clock_t_::time_point t_submit, t_done;
  bool done = false;
  int status = IFEAST_OK;
  std::string error;
  ifeast_result res{};
  std::vector<double> eval_re, eval_im, evec, resid, rf_hist;
  std::vector<int32_t> flags, inner_hist;
};

namespace {
// Requests whose solves allocate the same workspace (so a worker can keep it).
bool same_shape(const Request& a, const Request& b) {
  return a.n == b.n && a.hasB == b.hasB && a.C.nc == b.C.nc && a.p.m0 == b.p.m0 && a.p.max_inner == b.p.max_inner &&
         a.p.max_cycles == b.p.max_cycles && a.p.precision == b.p.precision && a.p.basis == b.p.basis &&
         a.p.problem == b.p.problem && a.footprint == b.footprint;
}
}  // namespace

Server::Server(ifeast_ctx* ctx) : ctx_(ctx) {
  for (int i = 0; i < kWorkers; ++i) workers_.emplace_back([this] { worker_loop(); });
}

Server::~Server() {
  std::unique_lock<std::mutex> lk(mu_);
  stop_ = true;
  // queued requests will not run: fail them and wake their waiters
  for (Request* r : queue_) {
    r->status = IFEAST_ERR_DEVICE;
    r->error = "context destroyed before the request ran";
    r->t_done = clock_t_::now();
    r->done = true;
  }
  queue_.clear();
  cv_.notify_all();
  lk.unlock();
  for (auto& t : workers_)
    if (t.joinable()) t.join();
  // running requests are done now; let every thread inside wait() leave before the state goes
  lk.lock();
  cv_.wait(lk, [this] { return waiters_ == 0; });
}

uint64_t Server::submit(const ifeast_csr* A, const ifeast_csr* B, const ifeast_contour& C, const ifeast_params& p,
                        const double* X0, uint64_t footprint) {
  std::unique_ptr<Request> r(new Request);
  r->footprint = footprint;
  r->n = A->n;
  r->rpA.assign(A->rowptr, A->rowptr + A->n + 1);
  r->ciA.assign(A->colind, A->colind + A->nnz);
  r->vA.assign(A->val, A->val + A->nnz);
  if (B) {
    r->hasB = true;
    r->rpB.assign(B->rowptr, B->rowptr + B->n + 1);
    r->ciB.assign(B->colind, B->colind + B->nnz);
    r->vB.assign(B->val, B->val + B->nnz);
  }
  r->C = C;
  if (C.kind == IFEAST_CONTOUR_EXPLICIT) {
    r->cz.assign(C.z, C.z + 2 * C.nc);
    r->cw.assign(C.w, C.w + 2 * C.nc);
    r->C.z = r->cz.data();
    r->C.w = r->cw.data();
  }
  r->p = p;
  if (X0) {
    r->hasX0 = true;
    r->X0.assign(X0, X0 + (size_t)A->n * p.m0);
  }
  r->t_submit = clock_t_::now();
  std::lock_guard<std::mutex> lk(mu_);
  if (stop_) throw Error{IFEAST_ERR_DEVICE, "the context is being destroyed"};
  r->ticket = next_++;
  const uint64_t t = r->ticket;
  queue_.push_back(r.get());
  all_[t] = std::move(r);
  cv_.notify_all();
  return t;
}

// The queue's front request fits next to the running ones (alone it always fits).
bool Server::admissible() const {
  return !queue_.empty() && (running_ == 0 || used_ + queue_.front()->footprint <= ctx_->budget);
}

void Server::worker_loop() {
  ifeast_ctx* sub = nullptr;  // this worker's stream and workspace
  std::unique_lock<std::mutex> lk(mu_);
  Request* r = nullptr;
  for (;;) {
    if (r == nullptr) {
      cv_.wait(lk, [this] { return stop_ || admissible(); });
      if (stop_) break;
      r = queue_.front();
      queue_.pop_front();
      used_ += r->footprint;
      ++running_;
    }
    lk.unlock();
    if (sub == nullptr && ifeast_create(&sub, ctx_->device, ctx_->budget) != IFEAST_OK) sub = nullptr;
    run(r, sub);
    lk.lock();
    r->t_done = clock_t_::now();
    r->done = true;
    Request* prev = r;
    r = nullptr;
    // the next queued request of the same shape reuses this worker's workspace: its footprint
    // replaces the finished one's
    if (!stop_ && !queue_.empty() && same_shape(*queue_.front(), *prev)) {
      r = queue_.front();
      queue_.pop_front();
    } else {
      used_ -= prev->footprint;
      --running_;
    }
    cv_.notify_all();
    if (r == nullptr && sub != nullptr) {
      lk.unlock();
      release_engine(sub);
      lk.lock();
    }
  }
  lk.unlock();
  if (sub != nullptr) ifeast_destroy(sub);
}

void Server::run(Request* r, ifeast_ctx* sub) {
  int status = IFEAST_OK;
  std::string err;
  const int m0 = r->p.m0;
  const bool general = r->p.problem == IFEAST_PROBLEM_GENERAL;
  r->eval_re.assign(m0, 0.0);
  r->eval_im.assign(m0, 0.0);
  r->resid.assign(m0, 0.0);
  r->flags.assign(m0, 0);
  r->evec.assign((size_t)r->n * m0 * (general ? 2 : 1), 0.0);
  r->rf_hist.assign(r->p.max_outer, 0.0);
  r->inner_hist.assign((size_t)r->p.max_outer * r->C.nc, 0);
  ifeast_result& res = r->res;
  res.eval_re = r->eval_re.data();
  res.eval_im = r->eval_im.data();
  res.resid = r->resid.data();
  res.flags = r->flags.data();
  res.evec = r->evec.data();
  res.rf_hist = r->rf_hist.data();
  res.inner_hist = r->inner_hist.data();
  if (sub != nullptr) {
    ifeast_csr A{r->n, (int64_t)r->ciA.size(), r->rpA.data(), r->ciA.data(), r->vA.data()};
    ifeast_csr B{r->n, (int64_t)r->ciB.size(), r->rpB.data(), r->ciB.data(), r->vB.data()};
    status = ifeast_solve(sub, &A, r->hasB ? &B : nullptr, &r->C, &r->p, r->hasX0 ? r->X0.data() : nullptr, &res);
    if (status < 0) err = ifeast_last_error(sub);
  } else {
    status = IFEAST_ERR_DEVICE;
    err = std::string("worker context: ") + ifeast_last_error(nullptr);
  }
  // free the request's inputs; keep the results
  std::vector<int64_t>().swap(r->rpA);
  std::vector<int32_t>().swap(r->ciA);
  std::vector<double>().swap(r->vA);
  std::vector<int64_t>().swap(r->rpB);
  std::vector<int32_t>().swap(r->ciB);
  std::vector<double>().swap(r->vB);
  std::vector<double>().swap(r->X0);
  std::lock_guard<std::mutex> lk(mu_);
  r->status = status;
  r->error = err;
}

int Server::poll(uint64_t ticket, int* done) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = all_.find(ticket);
  if (it == all_.end()) throw Error{IFEAST_ERR_UNKNOWN_TICKET, "unknown ticket"};
  *done = it->second->done ? 1 : 0;
  return IFEAST_OK;
}

int Server::wait(uint64_t ticket, ifeast_result* out, double* latency_s) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = all_.find(ticket);
  if (it == all_.end()) throw Error{IFEAST_ERR_UNKNOWN_TICKET, "unknown ticket"};
  Request* r = it->second.get();
  ++waiters_;
  cv_.wait(lk, [r] { return r->done; });
  const int m0 = r->p.m0;
  const ifeast_result& s = r->res;
  out->m = s.m;
  out->outer_iters = s.outer_iters;
  out->converged = s.converged;
  out->total_matvec = s.total_matvec;
  out->seq_matvec = s.seq_matvec;
  out->max_resid = s.max_resid;
  out->solve_seconds = s.solve_seconds;
  auto cp = [](auto* dst, const auto& src) {
    if (dst) std::copy(src.begin(), src.end(), dst);
  };
  cp(out->eval_re, r->eval_re);
  cp(out->eval_im, r->eval_im);
  cp(out->resid, r->resid);
  cp(out->flags, r->flags);
  cp(out->evec, r->evec);  // n x m0 (2 n x m0 interleaved complex for general problems)
  cp(out->rf_hist, r->rf_hist);
  cp(out->inner_hist, r->inner_hist);
  (void)m0;
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  const int status = r->status;
  // the error text goes to the context here, while the destructor still waits for this thread
  if (status < 0) ctx_->last_error = r->error;
  all_.erase(it);
  --waiters_;
  cv_.notify_all();
  return status;
}

}  // namespace ifeast
