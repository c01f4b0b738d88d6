// Continuous-batching server: requests are admitted as slots and HBM budget
// allow, every resident solve advances one outer iteration per step in the
// same launches (engine_step), finished solves retire at step boundaries and
// new ones join at the next step.  A solve's result does not depend on which
// other solves share its launches (per-job reductions, see common.h).
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>

#include "runtime.h"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Pending {
  int64_t ticket;
  dbl_request req;
  std::vector<double> psf;     // owned copy
  std::vector<double> sched;   // owned copy of mu_schedule
  double t_submit;
};

struct Finished {
  dbl_report rep;
};

}  // namespace

struct dbl_server {
  dbl_ctx* ctx = nullptr;
  int max_slots = 1;
  size_t budget = 0;
  size_t used = 0;
  int64_t next_ticket = 1;
  std::deque<std::unique_ptr<Pending>> queue;
  std::vector<std::unique_ptr<Pending>> resident_req;
  std::vector<std::unique_ptr<dbl::Slot>> resident;
  std::map<int64_t, Finished> finished;
};

namespace dbl {
int validate_request(dbl_ctx* ctx, const dbl_request& r);
}

using namespace dbl;

extern "C" {

int dbl_server_create(dbl_ctx* ctx, int max_slots, size_t budget, dbl_server** out) {
  if (!ctx || !out) return DBL_EINVAL;
  *out = nullptr;
  if (max_slots < 1 || max_slots > 4096) return set_err(ctx, DBL_EINVAL, "max_slots out of range");
  if (ctx->device < 0) return set_err(ctx, DBL_EDEVICE, "context has no device");
  dbl_server* s = new dbl_server();
  s->ctx = ctx;
  s->max_slots = max_slots;
  s->budget = budget;
  *out = s;
  return DBL_OK;
}

int dbl_server_destroy(dbl_server* srv) {
  if (!srv) return DBL_EINVAL;
  (void)hipStreamSynchronize(srv->ctx->stream);
  for (auto& sl : srv->resident) slot_free(srv->ctx, sl.get());
  delete srv;
  return DBL_OK;
}

int dbl_server_submit(dbl_server* srv, const dbl_request* req, int64_t* ticket) {
  if (!srv || !req || !ticket) return DBL_EINVAL;
  int rc = validate_request(srv->ctx, *req);
  if (rc) return rc;
  if (srv->budget && slot_bytes(*req) > srv->budget)
    return set_err(srv->ctx, DBL_ENOMEM, "request larger than the server budget");
  auto p = std::make_unique<Pending>();
  p->ticket = srv->next_ticket++;
  p->req = *req;
  p->psf.assign(req->psf, req->psf + (size_t)req->ph * req->pw);
  p->req.psf = p->psf.data();
  if (req->opts.mu_schedule) {
    p->sched.assign(req->opts.mu_schedule,
                    req->opts.mu_schedule + (size_t)req->levels * req->opts.k_out);
    p->req.opts.mu_schedule = p->sched.data();
  }
  p->t_submit = now_s();
  *ticket = p->ticket;
  srv->queue.push_back(std::move(p));
  return DBL_OK;
}

int dbl_server_step(dbl_server* srv, int* active) {
  if (!srv) return DBL_EINVAL;
  dbl_ctx* ctx = srv->ctx;
  (void)hipSetDevice(ctx->device);
  int rc = DBL_OK;
  // admit in arrival order while a slot and the budget allow
  while (!srv->queue.empty() && (int)srv->resident.size() < srv->max_slots) {
    Pending* p = srv->queue.front().get();
    const size_t bytes = slot_bytes(p->req);
    if (srv->budget && srv->used + bytes > srv->budget) break;
    auto sl = std::make_unique<Slot>();
    rc = slot_init(ctx, p->req, sl.get());
    if (rc) {
      slot_free(ctx, sl.get());
      // out of memory while other solves hold workspace: retry once they retire
      if (rc == DBL_ENOMEM && !srv->resident.empty()) break;
      // otherwise this request can never start: it finishes now with the
      // error as its status, and admission goes on with the next one
      Finished f;
      std::memset(&f.rep, 0, sizeof(f.rep));
      f.rep.levels = p->req.levels;
      f.rep.k_out = p->req.opts.k_out;
      f.rep.status = rc;
      f.rep.seconds = now_s() - p->t_submit;
      srv->finished[p->ticket] = f;
      srv->queue.pop_front();
      rc = DBL_OK;
      continue;
    }
    sl->ticket = p->ticket;
    sl->t_submit = p->t_submit;
    srv->used += bytes;
    srv->resident.push_back(std::move(sl));
    srv->resident_req.push_back(std::move(srv->queue.front()));
    srv->queue.pop_front();
  }
  if (!srv->resident.empty()) {
    std::vector<Slot*> ptrs;
    for (auto& sl : srv->resident) ptrs.push_back(sl.get());
    rc = engine_step(ctx, ptrs);
    if (rc) return rc;
    rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "server step");
    if (rc) return rc;
    const double t = now_s();
    for (size_t q = 0; q < srv->resident.size();) {
      Slot* sl = srv->resident[q].get();
      if (!sl->done) {
        ++q;
        continue;
      }
      Finished f;
      std::memset(&f.rep, 0, sizeof(f.rep));
      rc = slot_report(ctx, sl, &f.rep);
      if (rc) return rc;
      f.rep.seconds = t - sl->t_submit;
      // iterations a tolerance skipped are NaN by design; only run ones count
      for (int l = 0; l < sl->levels; ++l)
        for (int k = 0; k < f.rep.iters[l]; ++k)
          if (!std::isfinite(f.rep.objective[l][k])) f.rep.status = DBL_ENUMERIC;
      srv->finished[sl->ticket] = f;
      srv->used -= slot_bytes(sl->req);
      slot_free(ctx, sl);
      srv->resident.erase(srv->resident.begin() + q);
      srv->resident_req.erase(srv->resident_req.begin() + q);
    }
  }
  if (active) *active = (int)srv->resident.size();
  return DBL_OK;
}

int dbl_server_poll(dbl_server* srv, int64_t ticket, int* done, dbl_report* rep) {
  if (!srv || !done) return DBL_EINVAL;
  auto it = srv->finished.find(ticket);
  if (it != srv->finished.end()) {
    *done = 1;
    if (rep) *rep = it->second.rep;
    srv->finished.erase(it);
    return DBL_OK;
  }
  for (auto& p : srv->queue)
    if (p->ticket == ticket) {
      *done = 0;
      return DBL_OK;
    }
  for (auto& sl : srv->resident)
    if (sl->ticket == ticket) {
      *done = 0;
      return DBL_OK;
    }
  return set_err(srv->ctx, DBL_ENOTFOUND, "unknown ticket");
}

}  // extern "C"
