// Serving scheduler: continuous batching of deflated solves over several
// gauge fields (contexts), each field's eigenvector bank grown in place.
//
// Every registered context (field) gets a worker thread and a HIP stream of
// its own, so the work of different fields overlaps on the device.  Requests
// queue per field and are served in submission order:
//  * init-CG requests (EIGCG_MODE_INITCG) run as columns of a persistent
//    batched init-CG iteration over max_batch slots (a session, engine.cpp):
//    between iteration segments the worker retires finished slots (writing x
//    back) and admits waiting requests into free slots;
//  * eigCG requests (EIGCG_MODE_EIGCG, one step of Incremental eigCG,
//    Section 4) grow the field's bank: the worker lets the running slots
//    finish, solves the request with eigCG(nev, m) from its init-CG guess and
//    appends its Ritz vectors to the bank, so requests submitted after it are
//    deflated with the grown bank and those submitted before it with the
//    bank as it was.
// Admission is subject to the HBM budget: every context's resident memory
// (links, bank, work vectors, eigCG window once allocated) is charged once,
// every active init-CG request its working set, and an eigCG request the
// field's eigCG window while it is not yet allocated.  A small budget lowers
// the number of active slots (and makes an eigCG request wait for other
// fields' requests to finish); a request whose charge cannot fit even then
// fails with EIGCG_ENOMEM.  A request's arithmetic depends only on its own
// column and on the bank state its place in the field's queue fixes, so its
// result is the same alone and in the mix.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.h"


namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  uint64_t ticket = 0;
  int field = 0;
  int mode = EIGCG_MODE_INITCG;
  const void* b = nullptr;
  void* x = nullptr;
  double tol = 0.0;
  double t_submit = 0.0;
  double t_done = 0.0;
  bool done = false;
  eigcg_stats st{};
};

struct Field {
  eigcg_ctx* ctx = nullptr;
  hipStream_t own_stream = nullptr;
  hipStream_t saved_stream = nullptr;
  eigcg::Session* session = nullptr;
  std::deque<uint64_t> queue;
  size_t per_request = 0;  // working-set bytes charged per active init-CG request
  size_t resident = 0;     // the context's device bytes, as of its last operation
  size_t window = 0;       // eigCG window bytes while not yet allocated (0 after)
  int active = 0;          // active init-CG slots
  std::thread worker;
};

}  // namespace

struct eigcg_server {
  uint64_t budget = 0;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::vector<std::unique_ptr<Field>> fields;
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_ticket = 1;
  size_t outstanding = 0;
  bool stop = false;
  bool started = false;
  int error = 0;

  // bytes charged against the budget (caller holds mu)
  size_t charged() const {
    size_t b = 0;
    for (auto& f : fields) b += f->resident + f->per_request * (size_t)f->active;
    return b;
  }
  bool others_active(const Field* self) const {
    for (auto& f : fields)
      if (f.get() != self && f->active > 0) return true;
    return false;
  }

  // report finished requests (caller holds mu)
  void complete(const std::vector<eigcg::SessionDone>& done) {
    const double t = now_s();
    for (auto& d : done) {
      auto it = reqs.find(d.tag);
      if (it == reqs.end() || it->second.done) continue;
      Request& r = it->second;
      r.done = true;
      r.t_done = t;
      r.st.status = d.status;
      r.st.iters = d.iters;
      r.st.outer_steps = d.outer;
      r.st.first_leg_iters = d.first_leg;
      r.st.restart_tau = d.restart_tau;
      r.st.true_rel_res = d.true_rel_res;
      r.st.seconds = t - r.t_submit;
      --outstanding;
    }
    if (!done.empty()) cv_done.notify_all();
  }

  void fail_all(int code) {
    error = code;
    for (auto& kv : reqs)
      if (!kv.second.done) {
        kv.second.done = true;
        kv.second.st.status = code;
      }
    outstanding = 0;
    cv_done.notify_all();
    cv.notify_all();
  }

  // one eigCG request of field f, from the head of its queue (mu held on
  // entry and exit; the solve itself runs unlocked)
  void run_eigcg(Field& f, std::unique_lock<std::mutex>& lk) {
    const uint64_t t = f.queue.front();
    f.queue.pop_front();
    Request r = reqs[t];
    eigcg::Ctx& c = f.ctx->c;
    lk.unlock();
    eigcg_stats st{};
    int rc = EIGCG_OK;
    bool hip_failed = false;
    try {
      if (f.session) {  // the session's slots are idle; it reopens for the next init-CG
        eigcg::session_close(f.session);
        f.session = nullptr;
      }
      rc = eigcg::solve(c, 1, r.b, r.x, r.tol, EIGCG_MODE_EIGCG, &st);
    } catch (const eigcg::ApiError& e) {
      rc = e.code;
    } catch (...) {
      hip_failed = true;
    }
    lk.lock();
    f.resident = c.bytes;
    f.window = 0;
    if (hip_failed) {
      fail_all(EIGCG_EHIP);
      return;
    }
    eigcg::SessionDone d{};
    d.tag = t;
    d.status = rc;
    d.iters = st.iters;
    d.outer = st.outer_steps;
    d.first_leg = st.first_leg_iters;
    d.restart_tau = st.restart_tau;
    d.true_rel_res = st.true_rel_res;
    complete({d});
  }

  // field worker: serves the field's queue in order until the server stops
  void run_field(Field& f) {
    (void)hipSetDevice(f.ctx->c.device);
    std::unique_lock<std::mutex> lk(mu);
    while (!error) {
      cv.wait(lk, [&] { return stop || error || !f.queue.empty() || f.active > 0; });
      if (error || (stop && f.queue.empty() && f.active == 0)) break;
      std::vector<eigcg::SessionDone> done;
      const bool head_eig = !f.queue.empty() && reqs[f.queue.front()].mode == EIGCG_MODE_EIGCG;
      if (head_eig && f.active == 0) {
        // the window is charged while it is not yet allocated
        if (budget && charged() + f.window > budget) {
          if (others_active(&f)) {  // wait for other fields' requests to finish
            cv.wait_for(lk, std::chrono::milliseconds(2));
            continue;
          }
          const uint64_t t = f.queue.front();
          f.queue.pop_front();
          eigcg::SessionDone d{};
          d.tag = t;
          d.status = EIGCG_ENOMEM;
          complete({d});
          continue;
        }
        run_eigcg(f, lk);
        continue;
      }
      if (!f.session) {
        lk.unlock();
        bool ok = true;
        try {
          f.session = eigcg::session_open(f.ctx->c);
        } catch (...) {
          ok = false;
        }
        lk.lock();
        if (!ok) {
          fail_all(EIGCG_EHIP);
          break;
        }
        f.resident = f.ctx->c.bytes;
      }
      // admissions up to the next eigCG request (those wait for the slots to drain)
      while (!f.queue.empty() && reqs[f.queue.front()].mode != EIGCG_MODE_EIGCG &&
             eigcg::session_free_slot(f.session) >= 0) {
        if (budget && charged() + f.per_request > budget && f.active > 0) break;
        const uint64_t t = f.queue.front();
        Request r = reqs[t];
        f.queue.pop_front();
        lk.unlock();
        int slot = -1;
        bool hip_failed = false;
        try {
          slot = eigcg::session_admit(f.session, r.b, r.x, r.tol, t, done);
        } catch (const eigcg::ApiError& e) {
          eigcg::SessionDone d{};
          d.tag = t;
          d.status = e.code;
          done.push_back(d);
        } catch (...) {
          hip_failed = true;
        }
        lk.lock();
        if (hip_failed) {
          fail_all(EIGCG_EHIP);
          return;
        }
        f.active = eigcg::session_active(f.session);
        (void)slot;
      }
      // one iteration segment
      if (f.active > 0) {
        lk.unlock();
        bool hip_failed = false;
        try {
          eigcg::session_step(f.session, done);
        } catch (...) {
          hip_failed = true;
        }
        lk.lock();
        if (hip_failed) {
          fail_all(EIGCG_EHIP);
          return;
        }
        f.active = eigcg::session_active(f.session);
      }
      complete(done);
      if (!done.empty()) cv.notify_all();  // memory freed: other fields may admit
    }
  }

  void start() {
    started = true;
    for (auto& f : fields) {
      Field* fp = f.get();
      fp->worker = std::thread([this, fp] { run_field(*fp); });
    }
  }
};

extern "C" {

int eigcg_server_create(uint64_t hbm_budget, eigcg_server** out) {
  if (!out) return EIGCG_EINVAL;
  eigcg_server* s = new (std::nothrow) eigcg_server();
  if (!s) return EIGCG_ENOMEM;
  s->budget = hbm_budget;
  *out = s;
  return EIGCG_OK;
}

int eigcg_server_add(eigcg_server* srv, eigcg_ctx* ctx, int32_t* field_id) {
  if (!srv || !ctx) return EIGCG_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->started) return EIGCG_EINVAL;  // fields are registered before the first submit
  for (auto& f : srv->fields)
    if (f->ctx == ctx) return EIGCG_EINVAL;
  auto f = std::make_unique<Field>();
  f->ctx = ctx;
  f->saved_stream = ctx->c.stream;
  if (hipStreamCreateWithFlags(&f->own_stream, hipStreamNonBlocking) != hipSuccess)
    return EIGCG_EHIP;
  (void)hipStreamSynchronize(ctx->c.stream);
  ctx->c.stream = f->own_stream;
  eigcg::Ctx& c = ctx->c;
  // per-request working set: FP64 b, x, r, tmp (+ FP32 e, r, p, tmp when mixed;
  // FP32 e and 16-bit r, p, tmp in the half mode)
  const size_t v64 = c.cs * 16, v32 = c.cs * 8;
  const size_t v16 = c.cs * 4;
  f->per_request = 4 * v64 + (c.P.precision == EIGCG_MIXED_FP32 ? 4 * v32
                              : c.P.precision == EIGCG_MIXED_HALF ? v32 + 3 * v16 : v64);
  f->resident = c.bytes;
  f->window = eigcg::eig_window_bytes(c, 1);
  if (field_id) *field_id = (int32_t)srv->fields.size();
  srv->fields.push_back(std::move(f));
  return EIGCG_OK;
}

int eigcg_submit_mode(eigcg_server* srv, int32_t field_id, const void* b_dev, void* x_dev,
                      double tol, int32_t mode, uint64_t* ticket) {
  if (!srv || !b_dev || !x_dev || !ticket || !(tol > 0.0)) return EIGCG_EINVAL;
  if (mode != EIGCG_MODE_INITCG && mode != EIGCG_MODE_EIGCG) return EIGCG_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (field_id < 0 || field_id >= (int)srv->fields.size()) return EIGCG_EINVAL;
  if (srv->error) return srv->error;
  if (mode == EIGCG_MODE_EIGCG && srv->fields[field_id]->ctx->c.P.precision == EIGCG_MIXED_HALF)
    return EIGCG_EINVAL;  // eigCG needs FP64 or FP32 iterations
  if (!srv->started) srv->start();
  Request r;
  r.ticket = srv->next_ticket++;
  r.field = field_id;
  r.mode = mode;
  r.b = b_dev;
  r.x = x_dev;
  r.tol = tol;
  r.t_submit = now_s();
  srv->reqs[r.ticket] = r;
  srv->fields[field_id]->queue.push_back(r.ticket);
  ++srv->outstanding;
  *ticket = r.ticket;
  srv->cv.notify_all();
  return EIGCG_OK;
}

int eigcg_submit(eigcg_server* srv, int32_t field_id, const void* b_dev, void* x_dev, double tol,
                 uint64_t* ticket) {
  return eigcg_submit_mode(srv, field_id, b_dev, x_dev, tol, EIGCG_MODE_INITCG, ticket);
}

int eigcg_poll(eigcg_server* srv, uint64_t ticket, eigcg_stats* st) {
  if (!srv) return EIGCG_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return EIGCG_EINVAL;
  if (!it->second.done) return EIGCG_EBUSY;
  if (st) *st = it->second.st;
  return it->second.st.status;
}

int eigcg_server_drain(eigcg_server* srv) {
  if (!srv) return EIGCG_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->cv_done.wait(lk, [&] { return srv->outstanding == 0 || srv->error != 0; });
  return srv->error ? srv->error : EIGCG_OK;
}

int eigcg_server_destroy(eigcg_server* srv) {
  if (!srv) return EIGCG_EINVAL;
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->outstanding == 0 || srv->error != 0; });
    srv->stop = true;
    srv->cv.notify_all();
  }
  for (auto& f : srv->fields)
    if (f->worker.joinable()) f->worker.join();
  for (auto& f : srv->fields) {
    eigcg::session_close(f->session);
    (void)hipStreamSynchronize(f->own_stream);
    f->ctx->c.stream = f->saved_stream;
    (void)hipStreamDestroy(f->own_stream);
  }
  delete srv;
  return EIGCG_OK;
}

}  // extern "C"
