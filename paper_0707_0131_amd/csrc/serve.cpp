// Serving scheduler: continuous batching of deflated solves over several
// gauge fields (contexts).
//
// One worker thread owns all device work.  Each registered context gets a
// session (a persistent batched init-CG iteration over max_batch slots,
// engine.cpp) on its own HIP stream, so the iterations of different fields
// overlap on the device.  Requests queue per field; between iteration segments
// the worker retires finished slots (writing x back) and admits waiting
// requests into free slots, subject to the HBM budget: every context's
// resident memory (links, bank, work vectors) is charged once and every
// active request is charged its working set, so a small budget lowers the
// number of concurrently active slots without failing requests.  A request's
// arithmetic only depends on its own column (per-column reductions in a fixed
// order, per-column refinement schedule), so its result is the same alone
// and in the mix.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
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
  size_t per_request = 0;  // working-set bytes charged per active request
};

}  // namespace

struct eigcg_server {
  uint64_t budget = 0;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::vector<Field> fields;
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_ticket = 1;
  size_t outstanding = 0;
  bool stop = false;
  bool started = false;
  int error = 0;
  std::thread worker;

  size_t charged() {
    size_t b = 0;
    for (auto& f : fields) {
      b += f.ctx->c.bytes;
      if (f.session) b += f.per_request * (size_t)eigcg::session_active(f.session);
    }
    return b;
  }

  void run() {
    if (!fields.empty()) (void)hipSetDevice(fields[0].ctx->c.device);
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
      bool any = false;
      for (size_t fi = 0; fi < fields.size(); ++fi) {
        Field& f = fields[fi];
        if (!f.session && (!f.queue.empty())) {
          lk.unlock();
          try {
            f.session = eigcg::session_open(f.ctx->c);
          } catch (...) {
            error = EIGCG_EHIP;
          }
          lk.lock();
          if (!f.session) continue;
        }
        if (!f.session) continue;
        // admissions
        std::vector<eigcg::SessionDone> done;
        while (!f.queue.empty() && eigcg::session_free_slot(f.session) >= 0) {
          if (budget && charged() + f.per_request > budget && eigcg::session_active(f.session) > 0)
            break;
          const uint64_t t = f.queue.front();
          Request r = reqs[t];
          f.queue.pop_front();
          lk.unlock();
          int slot = -1;
          try {
            slot = eigcg::session_admit(f.session, r.b, r.x, r.tol, t, done);
          } catch (const eigcg::ApiError& e) {
            eigcg::SessionDone d{};
            d.tag = t;
            d.status = e.code;
            done.push_back(d);
          } catch (...) {
            error = EIGCG_EHIP;
          }
          lk.lock();
          (void)slot;
        }
        // one iteration segment
        if (eigcg::session_active(f.session) > 0) {
          any = true;
          lk.unlock();
          try {
            eigcg::session_step(f.session, done);
          } catch (...) {
            error = EIGCG_EHIP;
          }
          lk.lock();
        }
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
          r.st.true_rel_res = d.true_rel_res;
          r.st.seconds = t - r.t_submit;
          --outstanding;
        }
        if (!done.empty()) cv_done.notify_all();
        if (error) break;
      }
      if (error) {
        // fail every outstanding request
        for (auto& kv : reqs)
          if (!kv.second.done) {
            kv.second.done = true;
            kv.second.st.status = error;
          }
        outstanding = 0;
        cv_done.notify_all();
        break;
      }
      if (!any) {
        bool queued = false;
        for (auto& f : fields) queued = queued || !f.queue.empty();
        if (!queued) cv.wait(lk, [&] {
          if (stop) return true;
          for (auto& f : fields)
            if (!f.queue.empty()) return true;
          return false;
        });
      }
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
    if (f.ctx == ctx) return EIGCG_EINVAL;
  Field f;
  f.ctx = ctx;
  f.saved_stream = ctx->c.stream;
  if (hipStreamCreateWithFlags(&f.own_stream, hipStreamNonBlocking) != hipSuccess)
    return EIGCG_EHIP;
  (void)hipStreamSynchronize(ctx->c.stream);
  ctx->c.stream = f.own_stream;
  // per-request working set: FP64 b, x, r, tmp (+ FP32 e, r, p, tmp when mixed;
  // FP32 e and 16-bit r, p, tmp in the half mode)
  const size_t v64 = ctx->c.cs * 16, v32 = ctx->c.cs * 8;
  const size_t v16 = ctx->c.cs * 4;
  f.per_request = 4 * v64 + (ctx->c.P.precision == EIGCG_MIXED_FP32 ? 4 * v32
                             : ctx->c.P.precision == EIGCG_MIXED_HALF ? v32 + 3 * v16 : v64);
  if (field_id) *field_id = (int32_t)srv->fields.size();
  srv->fields.push_back(f);
  return EIGCG_OK;
}

int eigcg_submit(eigcg_server* srv, int32_t field_id, const void* b_dev, void* x_dev, double tol,
                 uint64_t* ticket) {
  if (!srv || !b_dev || !x_dev || !ticket || !(tol > 0.0)) return EIGCG_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (field_id < 0 || field_id >= (int)srv->fields.size()) return EIGCG_EINVAL;
  if (srv->error) return srv->error;
  if (!srv->started) {
    srv->started = true;
    srv->worker = std::thread([srv] { srv->run(); });
  }
  Request r;
  r.ticket = srv->next_ticket++;
  r.field = field_id;
  r.b = b_dev;
  r.x = x_dev;
  r.tol = tol;
  r.t_submit = now_s();
  srv->reqs[r.ticket] = r;
  srv->fields[field_id].queue.push_back(r.ticket);
  ++srv->outstanding;
  *ticket = r.ticket;
  srv->cv.notify_all();
  return EIGCG_OK;
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
  if (srv->worker.joinable()) srv->worker.join();
  for (auto& f : srv->fields) {
    eigcg::session_close(f.session);
    (void)hipStreamSynchronize(f.own_stream);
    f.ctx->c.stream = f.saved_stream;
    (void)hipStreamDestroy(f.own_stream);
  }
  delete srv;
  return EIGCG_OK;
}

}  // extern "C"
