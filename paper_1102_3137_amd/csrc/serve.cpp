// Request server: asynchronous Dyson solves with continuous batching.
//
// Frequencies are independent problems (each H(i w_k) is solved on its own;
// Sec. I), so a request is cut into runs of frequencies.  A pool of slots,
// each a host thread with its own HIP stream and workspace, forms a batch
// from the oldest waiting frequencies plus those of every other waiting
// request on the same plan, as many as the HBM budget and the batch cap
// allow, and runs the whole hot path on it.  Requests that arrive while
// batches are on the device are taken by the next slot that frees up, and
// the slots' batches overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/dyson.h"
#include "engine.h"

using namespace dyson;
using Clock = std::chrono::steady_clock;

namespace dyson {

struct ReqState {
  dyson_plan* plan = nullptr;
  int K = 0, mem = DYSON_MEM_DEVICE;
  int zmode = 0;  // 0: omega holds Matsubara w_k; 1: complex energies z_k
  const double *V = nullptr, *omega = nullptr, *sigma = nullptr;  // device mode
  double* G = nullptr;                                             // caller's output
  std::vector<double> hV, hom, hsig;                               // host mode copies
  // guarded by Server::m
  int next_k = 0;    // first frequency not yet handed to a slot
  int running = 0;   // batches holding some of its frequencies
  bool finished = false, started = false;
  dyson_status status = DYSON_OK;
  std::string err;
  Clock::time_point t_arrive, t_start, t_end;
  dyson_report agg{};
  std::atomic<bool> cancelled{false};
};

struct Piece {
  std::shared_ptr<ReqState> r;
  int k0, n;
};

struct Slot {
  Work work;
  hipStream_t stream = nullptr;
  bool busy = false;
  std::thread th;
};

struct Server {
  dyson_ctx* ctx = nullptr;
  int device = 0;
  size_t budget = 0;
  int max_batch = 256;
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<ReqState>> queue;  // requests with frequencies not yet taken
  std::vector<std::unique_ptr<Slot>> slots;
  size_t reserved = 0;      // device bytes held by slot workspaces
  unsigned long long gen = 0;  // bumped whenever memory or the queue changes
  bool stop = false;
  bool joined = false;
  // input validation of device-mode submissions
  std::mutex vm;
  hipStream_t vstream = nullptr;
  int* vflag = nullptr;
  int* hflag = nullptr;

  void finish_locked(ReqState& r) {
    r.finished = true;
    r.t_end = Clock::now();
    if (!r.started) r.t_start = r.t_end;
    if (r.cancelled.load() && r.status == DYSON_OK) {
      r.status = DYSON_ECANCELLED;
      r.err = "request cancelled";
    }
    cv_done.notify_all();
  }

  void cancel_locked(const std::shared_ptr<ReqState>& r) {
    if (r->finished) return;
    r->cancelled.store(true);
    auto it = std::find(queue.begin(), queue.end(), r);
    if (it != queue.end()) queue.erase(it);
    r->next_k = r->K;
    if (r->running == 0) finish_locked(*r);
    ++gen;
    cv_work.notify_all();
  }

  void fail_locked(const std::shared_ptr<ReqState>& r, dyson_status st, const std::string& msg) {
    auto it = std::find(queue.begin(), queue.end(), r);
    if (it != queue.end()) queue.erase(it);
    r->next_k = r->K;
    if (r->status == DYSON_OK) {
      r->status = st;
      r->err = msg;
    }
    if (r->running == 0) finish_locked(*r);
  }

  // Largest K <= want whose workspace fits in `room` bytes (0 if none).
  int fit(const dyson_plan* p, int want, size_t room) const {
    if (work_bytes(p, 1) > room) return 0;
    int lo = 1, hi = want;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (work_bytes(p, mid) <= room) lo = mid;
      else hi = mid - 1;
    }
    return lo;
  }

  enum Formed { BATCH, WAIT, RETRY };

  // Under m: take frequencies for slot si.  Sets *realloc when the slot's
  // workspace has to be (re)allocated for kb frequencies of the plan.
  Formed form(int si, std::vector<Piece>& pieces, int* kb_out, bool* realloc) {
    Slot& sl = *slots[si];
    const std::shared_ptr<ReqState> head = queue.front();
    dyson_plan* P = head->plan;
    long long want = 0;
    for (auto& r : queue)
      if (r->plan == P) want += r->K - r->next_k;
    const int w = (int)std::min<long long>(want, max_batch);
    int kb = 0;
    *realloc = false;
    if (sl.work.plan == P && sl.work.Kcap >= w) {
      kb = w;
    } else {
      const size_t held = reserved - sl.work.bytes;
      kb = budget > held ? fit(P, w, budget - held) : 0;
      if (sl.work.plan == P && sl.work.Kcap >= kb) kb = std::min(w, sl.work.Kcap);
      else *realloc = kb > 0;
      if (kb == 0) {
        // give back the workspaces of idle slots and try again
        bool freed = false;
        for (auto& o : slots)
          if (!o->busy && o.get() != &sl && o->work.bytes) {
            reserved -= o->work.bytes;
            free_work(&o->work, o->stream);
            freed = true;
          }
        if (freed) return RETRY;
        bool any_busy = false;
        for (auto& o : slots) any_busy |= o->busy;
        if (any_busy) return WAIT;
        fail_locked(head, DYSON_ENOMEM,
                    "one frequency of this plan needs " + std::to_string(work_bytes(P, 1)) +
                        " device bytes, more than the serving budget of " +
                        std::to_string(budget));
        return RETRY;
      }
    }
    if (*realloc) {
      reserved -= sl.work.bytes;
      reserved += work_bytes(P, kb);
    }
    int taken = 0;
    const auto now = Clock::now();
    for (size_t i = 0; i < queue.size() && taken < kb;) {
      auto r = queue[i];
      if (r->plan != P) {
        ++i;
        continue;
      }
      const int c = std::min(r->K - r->next_k, kb - taken);
      pieces.push_back(Piece{r, r->next_k, c});
      r->next_k += c;
      r->running += 1;
      if (!r->started) {
        r->started = true;
        r->t_start = now;
      }
      taken += c;
      if (r->next_k == r->K) queue.erase(queue.begin() + i);
      else ++i;
    }
    *kb_out = kb;
    sl.busy = true;
    return BATCH;
  }

  // Runs one batch on slot si (no lock held).
  dyson_status run(int si, const std::vector<Piece>& pieces, int kb, bool realloc,
                   dyson_report* rep) {
    Slot& sl = *slots[si];
    dyson_plan* P = pieces[0].r->plan;
    if (hipSetDevice(device) != hipSuccess) {
      set_error("hipSetDevice failed");
      return DYSON_EDEVICE;
    }
    if (realloc) {
      dyson_status st = ensure_work(P, &sl.work, kb, sl.stream);
      if (st != DYSON_OK) return st;
    }
    Work* w = &sl.work;
    const int N = P->hp.N;
    const size_t NP = (size_t)P->hp.T * P->hp.S;
    std::vector<Slice> slices;
    int k0 = 0;
    for (size_t j = 0; j < pieces.size(); ++j) {
      const Piece& pc = pieces[j];
      ReqState& r = *pc.r;
      const int zw = r.zmode ? 2 : 1;  // doubles per frequency
      Slice s{pc.n, nullptr, nullptr, nullptr, nullptr, r.zmode};
      if (r.mem == DYSON_MEM_DEVICE) {
        s.V = r.V;
        s.omega = r.omega + (size_t)pc.k0 * zw;
        s.sigma = r.sigma + (size_t)pc.k0 * N * 2;
        s.G = r.G + (size_t)pc.k0 * N * 2;
      } else {
        // staging: V rows in r, frequencies in stage_om, Sigma in the rows
        // of xB that the batch's G will later be scattered to (xB is free
        // before the first correction level and after the last)
        double* sv = w->r + (size_t)j * N;
        double* so = w->stage_om + 2 * (size_t)k0;
        double* ss = w->xB + (size_t)k0 * NP * 2;
        if (hipMemcpyAsync(sv, r.hV.data(), (size_t)N * 8, hipMemcpyHostToDevice, sl.stream) !=
                hipSuccess ||
            hipMemcpyAsync(so, r.hom.data() + (size_t)pc.k0 * zw, (size_t)pc.n * zw * 8,
                           hipMemcpyHostToDevice, sl.stream) != hipSuccess ||
            hipMemcpyAsync(ss, r.hsig.data() + (size_t)pc.k0 * N * 2, (size_t)pc.n * N * 16,
                           hipMemcpyHostToDevice, sl.stream) != hipSuccess) {
          set_error("host to device copy failed");
          return DYSON_EDEVICE;
        }
        s.V = sv;
        s.omega = so;
        s.sigma = ss;
        s.G = ss;
      }
      slices.push_back(s);
      k0 += pc.n;
    }
    auto abort = [&pieces] {
      for (auto& pc : pieces)
        if (!pc.r->cancelled.load()) return false;
      return true;
    };
    dyson_status st =
        run_solve(P, w, slices.data(), (int)slices.size(), sl.stream, rep, abort);
    if (st != DYSON_OK) return st;
    for (size_t j = 0; j < pieces.size(); ++j) {
      ReqState& r = *pieces[j].r;
      if (r.mem != DYSON_MEM_HOST || r.cancelled.load()) continue;
      if (hipMemcpyAsync(r.G + (size_t)pieces[j].k0 * N * 2, slices[j].G,
                         (size_t)pieces[j].n * N * 16, hipMemcpyDeviceToHost,
                         sl.stream) != hipSuccess) {
        set_error("device to host copy failed");
        return DYSON_EDEVICE;
      }
    }
    if (hipStreamSynchronize(sl.stream) != hipSuccess) {
      set_error("stream synchronize failed");
      return DYSON_EDEVICE;
    }
    return DYSON_OK;
  }

  void worker(int si) {
    (void)hipSetDevice(device);
    Slot& sl = *slots[si];
    std::unique_lock<std::mutex> lk(m);
    for (;;) {
      cv_work.wait(lk, [&] { return stop || !queue.empty(); });
      if (stop) break;
      std::vector<Piece> pieces;
      int kb = 0;
      bool realloc = false;
      const unsigned long long g0 = gen;
      const Formed f = form(si, pieces, &kb, &realloc);
      if (f == RETRY) continue;
      if (f == WAIT) {
        cv_work.wait(lk, [&] { return stop || gen != g0; });
        continue;
      }
      lk.unlock();
      dyson_report rep{};
      dyson_status st = run(si, pieces, kb, realloc, &rep);
      const std::string msg = st == DYSON_OK ? std::string() : get_error();
      lk.lock();
      if (realloc) {  // the reservation assumed the allocation succeeded
        reserved -= work_bytes(pieces[0].r->plan, kb);
        reserved += sl.work.bytes;
      }
      for (auto& pc : pieces) {
        ReqState& r = *pc.r;
        r.running -= 1;
        // a failed batch fails its requests; their queued frequencies are dropped
        if (st != DYSON_OK && st != DYSON_ECANCELLED) fail_locked(pc.r, st, msg);
        dyson_report& a = r.agg;
        a.batches += 1;
        a.levels = rep.levels;
        a.max_rank_used = std::max(a.max_rank_used, rep.max_rank_used);
        a.lanczos_steps += rep.lanczos_steps;
        a.inner_iters += rep.inner_iters;
        a.inner_iters_max = std::max(a.inner_iters_max, rep.inner_iters_max);
        a.restarts += rep.restarts;
        a.truncated |= rep.truncated;
        a.hbm_bytes = std::max(a.hbm_bytes, sl.work.bytes);
        // the batch's check covers every frequency in it, this request's too
        if (st == DYSON_OK)
          a.est_rel_err = (rep.est_rel_err != rep.est_rel_err || a.est_rel_err != a.est_rel_err)
                              ? std::nan("")
                              : std::max(a.est_rel_err, rep.est_rel_err);
        for (int c = 0; c < 4; ++c) {
          a.kern_ms[c] += rep.kern_ms[c];
          a.kern_launches[c] += rep.kern_launches[c];
          a.kern_bytes[c] += rep.kern_bytes[c];
        }
        if (r.running == 0 && r.next_k == r.K && !r.finished) finish_locked(r);
      }
      sl.busy = false;
      ++gen;
      cv_work.notify_all();
    }
  }

  void shutdown() {
    {
      std::lock_guard<std::mutex> g(m);
      if (joined) return;
      stop = true;
      auto q = queue;
      for (auto& r : q) cancel_locked(r);
      queue.clear();
      cv_work.notify_all();
    }
    for (auto& s : slots)
      if (s->th.joinable()) s->th.join();
    (void)hipSetDevice(device);
    for (auto& s : slots) {
      free_work(&s->work, s->stream);
      if (s->stream) (void)hipStreamDestroy(s->stream);
      s->stream = nullptr;
    }
    if (vstream) (void)hipStreamDestroy(vstream);
    if (vflag) (void)hipFree(vflag);
    if (hflag) (void)hipHostFree(hflag);
    vstream = nullptr;
    vflag = hflag = nullptr;
    joined = true;
  }
};

void serve_forget_plan(dyson_ctx* c, const dyson_plan* p) {
  std::shared_ptr<Server> srv;
  {
    std::lock_guard<std::mutex> g(c->server_mu);
    srv = c->server;
  }
  if (!srv) return;
  std::lock_guard<std::mutex> g(srv->m);
  for (auto& s : srv->slots)
    if (!s->busy && s->work.plan == p) {
      srv->reserved -= s->work.bytes;
      free_work(&s->work, s->stream);
    }
  ++srv->gen;
  srv->cv_work.notify_all();
}

}  // namespace dyson

dyson_ctx::~dyson_ctx() {
  std::shared_ptr<Server> srv;
  {
    std::lock_guard<std::mutex> g(server_mu);
    srv = server;
    server.reset();
  }
  if (srv) srv->shutdown();
}

struct dyson_req {
  std::shared_ptr<Server> srv;
  std::shared_ptr<ReqState> st;
};

namespace {

dyson_status fail(dyson_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

dyson_status start_server(dyson_ctx* c, std::shared_ptr<Server>* out) {
  std::lock_guard<std::mutex> g(c->server_mu);
  if (c->server) {
    *out = c->server;
    return DYSON_OK;
  }
  if (hipSetDevice(c->device) != hipSuccess) return fail(DYSON_EDEVICE, "hipSetDevice failed");
  auto srv = std::make_shared<Server>();
  srv->ctx = c;
  srv->device = c->device;
  srv->budget = c->budget;
  srv->max_batch = c->max_batch_freqs;
  if (hipStreamCreateWithFlags(&srv->vstream, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc((void**)&srv->vflag, sizeof(int)) != hipSuccess ||
      hipHostMalloc((void**)&srv->hflag, sizeof(int), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    srv->shutdown();
    return fail(DYSON_EDEVICE, "could not create the server's validation stream");
  }
  for (int i = 0; i < c->slots; ++i) {
    auto s = std::make_unique<Slot>();
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      srv->slots.push_back(std::move(s));
      srv->shutdown();
      return fail(DYSON_EDEVICE, "could not create a slot stream");
    }
    srv->slots.push_back(std::move(s));
  }
  Server* raw = srv.get();
  for (int i = 0; i < c->slots; ++i) srv->slots[i]->th = std::thread([raw, i] { raw->worker(i); });
  c->server = srv;
  *out = srv;
  return DYSON_OK;
}

const char* kMixed16Msg =
    "DYSON_PREC_MIXED16 needs Im(z_k - Sigma_i) >= 2^-14: its FP16 factor entries reach "
    "1 / min Im H_ii; use DYSON_PREC_MIXED or DYSON_PREC_FP64";

dyson_status validate_host(int N, int K, const double* V, const double* om, int zmode,
                           const double* sg, double min_im) {
  for (int i = 0; i < N; ++i)
    if (!std::isfinite(V[i])) return fail(DYSON_EINVAL, "V contains a non-finite value");
  for (int k = 0; k < K; ++k) {
    const double zr = zmode ? om[2 * k] : 0.0, zi = zmode ? om[2 * k + 1] : om[k];
    if (!std::isfinite(zr) || !std::isfinite(zi) || !(zi > 0))
      return fail(DYSON_EINVAL, "frequencies must be finite with w_k > 0 (Im z_k > 0)");
    for (int i = 0; i < N; ++i) {
      const double re = sg[2 * ((size_t)k * N + i)], im = sg[2 * ((size_t)k * N + i) + 1];
      if (!std::isfinite(re) || !std::isfinite(im))
        return fail(DYSON_EINVAL, "Sigma contains a non-finite value");
      if (!(zi - im > 0))
        return fail(DYSON_EINVAL, "Im(z_k - Sigma_i) must be > 0 (causal self-energy)");
      if (zi - im < min_im) return fail(DYSON_EUNSUPPORTED, kMixed16Msg);
    }
  }
  return DYSON_OK;
}

dyson_status validate_device(Server& srv, int N, int K, const double* V, const double* om,
                             int zmode, const double* sg, double min_im) {
  std::lock_guard<std::mutex> g(srv.vm);
  if (hipSetDevice(srv.device) != hipSuccess)
    return fail(DYSON_EDEVICE, "validation launch failed");
  launch_zero(srv.vflag, sizeof(int), srv.vstream);
  // frequencies index the second grid dimension: at most 65535 per launch
  for (int k0 = 0; k0 < K; k0 += 65535) {
    const int kn = std::min(K - k0, 65535);
    launch_validate(N, kn, V, om + (size_t)k0 * (zmode ? 2 : 1), zmode,
                    sg + (size_t)k0 * N * 2, min_im, srv.vflag, srv.vstream);
  }
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(srv.hflag, srv.vflag, sizeof(int), hipMemcpyDeviceToHost, srv.vstream) !=
          hipSuccess ||
      hipStreamSynchronize(srv.vstream) != hipSuccess)
    return fail(DYSON_EDEVICE, "validation kernel failed");
  const int f = *srv.hflag;
  if (f & 1) return fail(DYSON_EINVAL, "V contains a non-finite value");
  if (f & 2) return fail(DYSON_EINVAL, "frequencies must be finite with w_k > 0 (Im z_k > 0)");
  if (f & 4) return fail(DYSON_EINVAL, "Sigma contains a non-finite value");
  if (f & 8) return fail(DYSON_EINVAL, "Im(z_k - Sigma_i) must be > 0 (causal self-energy)");
  if (f & 16) return fail(DYSON_EUNSUPPORTED, kMixed16Msg);
  return DYSON_OK;
}

}  // namespace

namespace {

dyson_status submit(dyson_plan* plan, int K, const double* V, const double* omega, int zmode,
                    const double* sigma, double* G, int mem, dyson_req** req) {
  if (!plan || !plan->ctx) return fail(DYSON_EINVAL, "plan has no device context");
  if (!req) return fail(DYSON_EINVAL, "null request handle");
  if (K < 1) return fail(DYSON_EINVAL, "K must be >= 1");
  if (!V || !omega || !sigma || !G) return fail(DYSON_EINVAL, "null input or output pointer");
  if (mem != DYSON_MEM_DEVICE && mem != DYSON_MEM_HOST) return fail(DYSON_EINVAL, "bad mem");
  std::shared_ptr<Server> srv;
  dyson_status s0 = start_server(plan->ctx, &srv);
  if (s0 != DYSON_OK) return s0;
  const int N = plan->hp.N;
  const double min_im = plan->hp.opts.precision == DYSON_PREC_MIXED16 ? kMinImMixed16 : 0.0;
  auto r = std::make_shared<ReqState>();
  r->plan = plan;
  r->K = K;
  r->mem = mem;
  r->zmode = zmode;
  r->G = G;
  if (mem == DYSON_MEM_HOST) {
    dyson_status sv = validate_host(N, K, V, omega, zmode, sigma, min_im);
    if (sv != DYSON_OK) return sv;
    r->hV.assign(V, V + N);
    r->hom.assign(omega, omega + (size_t)K * (zmode ? 2 : 1));
    r->hsig.assign(sigma, sigma + (size_t)2 * K * N);
  } else {
    dyson_status sv = validate_device(*srv, N, K, V, omega, zmode, sigma, min_im);
    if (sv != DYSON_OK) return sv;
    r->V = V;
    r->omega = omega;
    r->sigma = sigma;
  }
  r->t_arrive = Clock::now();
  plan->live_requests.fetch_add(1);
  {
    std::lock_guard<std::mutex> g(srv->m);
    if (srv->stop) {
      plan->live_requests.fetch_sub(1);
      return fail(DYSON_EINVAL, "the context is being destroyed");
    }
    srv->queue.push_back(r);
    ++srv->gen;
  }
  srv->cv_work.notify_all();
  *req = new dyson_req{srv, r};
  return DYSON_OK;
}

}  // namespace

extern "C" {

dyson_status dyson_serve_config(dyson_ctx* ctx, int slots, int max_batch_freqs) {
  if (!ctx) return fail(DYSON_EINVAL, "null ctx");
  if (slots < 1 || slots > 8) return fail(DYSON_EINVAL, "slots must be in [1, 8]");
  if (max_batch_freqs < 1 || max_batch_freqs > 4096)
    return fail(DYSON_EINVAL, "max_batch_freqs must be in [1, 4096]");
  std::lock_guard<std::mutex> g(ctx->server_mu);
  if (ctx->server) return fail(DYSON_EBUSY, "the server has already started");
  ctx->slots = slots;
  ctx->max_batch_freqs = max_batch_freqs;
  return DYSON_OK;
}

dyson_status dyson_submit(dyson_plan* plan, int K, const double* V, const double* omega,
                          const double* sigma, double* G, int mem, dyson_req** req) {
  return submit(plan, K, V, omega, 0, sigma, G, mem, req);
}

dyson_status dyson_submit_z(dyson_plan* plan, int K, const double* V, const double* z,
                            const double* sigma, double* G, int mem, dyson_req** req) {
  return submit(plan, K, V, z, 1, sigma, G, mem, req);
}

dyson_status dyson_poll(dyson_req* req, int* done) {
  if (!req || !done) return fail(DYSON_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(req->srv->m);
  *done = req->st->finished ? 1 : 0;
  return DYSON_OK;
}

dyson_status dyson_wait(dyson_req* req, double timeout_s) {
  if (!req) return fail(DYSON_EINVAL, "null request");
  Server& srv = *req->srv;
  ReqState& r = *req->st;
  std::unique_lock<std::mutex> lk(srv.m);
  auto pred = [&] { return r.finished; };
  if (timeout_s < 0) {
    srv.cv_done.wait(lk, pred);
  } else if (!srv.cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
    return fail(DYSON_ETIMEOUT, "request not finished within the timeout");
  }
  if (r.status != DYSON_OK) set_error(r.err);
  return r.status;
}

dyson_status dyson_cancel(dyson_req* req) {
  if (!req) return fail(DYSON_EINVAL, "null request");
  std::lock_guard<std::mutex> g(req->srv->m);
  req->srv->cancel_locked(req->st);
  return DYSON_OK;
}

dyson_status dyson_req_report(dyson_req* req, dyson_report* rep) {
  if (!req || !rep) return fail(DYSON_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(req->srv->m);
  const ReqState& r = *req->st;
  if (!r.finished) return fail(DYSON_EBUSY, "request not finished");
  *rep = r.agg;
  rep->t_total_ms = std::chrono::duration<double, std::milli>(r.t_end - r.t_arrive).count();
  rep->t_queue_ms = std::chrono::duration<double, std::milli>(r.t_start - r.t_arrive).count();
  return DYSON_OK;
}

dyson_status dyson_release(dyson_req* req) {
  if (!req) return DYSON_OK;
  {
    std::unique_lock<std::mutex> lk(req->srv->m);
    req->srv->cancel_locked(req->st);
    req->srv->cv_done.wait(lk, [&] { return req->st->running == 0; });
  }
  req->st->plan->live_requests.fetch_sub(1);
  delete req;
  return DYSON_OK;
}

dyson_status dyson_solve_batch(int n, dyson_plan* const* plans, const int* Ks,
                               const double* const* d_V, const double* const* d_omega,
                               const double* const* d_sigma, double* const* d_G, void* stream,
                               dyson_report* reports) {
  if (n < 1 || !plans || !Ks || !d_V || !d_omega || !d_sigma || !d_G)
    return fail(DYSON_EINVAL, "bad batch arguments");
  dyson_ctx* ctx = plans[0] ? plans[0]->ctx : nullptr;
  for (int i = 0; i < n; ++i)
    if (!plans[i] || plans[i]->ctx != ctx || !ctx)
      return fail(DYSON_EINVAL, "every plan of a batch must belong to one context");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(DYSON_EDEVICE, "hipSetDevice failed");
  // the inputs are read on the server's streams: complete them first
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return fail(DYSON_EDEVICE, "caller stream failed");
  std::vector<dyson_req*> reqs(n, nullptr);
  dyson_status st = DYSON_OK;
  std::string err;
  for (int i = 0; i < n && st == DYSON_OK; ++i) {
    st = submit(plans[i], Ks[i], d_V[i], d_omega[i], 0, d_sigma[i], d_G[i], DYSON_MEM_DEVICE,
                &reqs[i]);
    if (st != DYSON_OK) err = get_error();
  }
  for (int i = 0; i < n; ++i) {
    if (!reqs[i]) continue;
    if (st != DYSON_OK) {
      (void)dyson_release(reqs[i]);  // cancels what has not started
      continue;
    }
    const dyson_status si = dyson_wait(reqs[i], -1.0);
    if (si != DYSON_OK && st == DYSON_OK) {
      st = si;
      err = get_error();
    }
    if (reports) (void)dyson_req_report(reqs[i], &reports[i]);
    (void)dyson_release(reqs[i]);
  }
  if (st != DYSON_OK) return fail(st, err);
  return DYSON_OK;
}

}  // extern "C"
