// Host-only check of the request server (serve.cpp) under ThreadSanitizer or
// AddressSanitizer + UndefinedBehaviorSanitizer, built by
// tests/test_native_sanitizers.py with g++ against tests/native/stub (a host
// stand-in for the HIP runtime).  serve.cpp and the planner are the library's
// own sources; the device layer below them (workspace sizing and allocation,
// input validation, the solve itself) is replaced by host code.  The stand-in
// solve writes a closed function of each (frequency, site) input,
// G = 1 / (z_k + mu - V_i - Sigma_i(z_k)), so the result of every request is
// known exactly whatever batches its frequencies ran in: the check drives
// several submitting threads, both memory modes, both energy kinds, cancels,
// timeouts, invalid inputs, a budget that splits requests into many batches
// and dyson_solve_batch, and compares every finished G bit for bit.
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../include/dyson.h"
#include "../../paper_1102_3137_amd/csrc/engine.h"

using namespace dyson;

// ------------------------------------------------ HIP runtime stand-in
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipMalloc(void** p, size_t n) {
  *p = std::malloc(n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { return hipMalloc(p, n); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  std::memcpy(d, s, n);
  return hipSuccess;
}
struct ihipStream_t {
  int id;
};
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new ihipStream_t{0};
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }

// ------------------------------------------------ device layer stand-in
namespace dyson {
const double kMinImMixed16 = 1.0 / 16384.0;
static thread_local std::string t_err;
void set_error(const std::string& m) { t_err = m; }
const std::string& get_error() { return t_err; }
Prof::~Prof() {}

// bytes per frequency of a workspace: small enough that a few frequencies fit
// in the check's budget, so requests are cut into several batches
size_t work_bytes(const dyson_plan* p, int K) {
  return (size_t)K * ((size_t)p->hp.N + (size_t)p->hp.T * p->hp.S) * 64;
}

static void release_buffers(Work* w) {
  std::free(w->r);
  std::free(w->stage_om);
  std::free(w->xB);
  w->r = w->stage_om = w->xB = nullptr;
}

dyson_status ensure_work(const dyson_plan* p, Work* w, int K, hipStream_t) {
  if (w->plan == p && w->Kcap >= K) return DYSON_OK;
  release_buffers(w);
  const size_t N = p->hp.N, NP = (size_t)p->hp.T * p->hp.S;
  // the server stages host-mode inputs in r (one V row per piece), stage_om
  // and xB (the batch's Sigma, then its G)
  w->r = (double*)std::calloc((size_t)K * N, sizeof(double));
  w->stage_om = (double*)std::calloc(2 * (size_t)K, sizeof(double));
  w->xB = (double*)std::calloc((size_t)K * NP * 2, sizeof(double));
  if (!w->r || !w->stage_om || !w->xB) {
    release_buffers(w);
    w->plan = nullptr;
    w->Kcap = 0;
    w->bytes = 0;
    set_error("workspace allocation failed");
    return DYSON_ENOMEM;
  }
  w->plan = p;
  w->Kcap = K;
  w->bytes = work_bytes(p, K);
  return DYSON_OK;
}

void free_work(Work* w, hipStream_t) {
  release_buffers(w);
  w->plan = nullptr;
  w->Kcap = 0;
  w->bytes = 0;
}

void launch_zero(void* p, size_t bytes, hipStream_t) { std::memset(p, 0, bytes); }

void launch_validate(int N, int K, const double* V, const double* om, int zmode,
                     const double* sg, double min_im, int* flag, hipStream_t) {
  int f = 0;
  for (int i = 0; i < N; ++i)
    if (!std::isfinite(V[i])) f |= 1;
  for (int k = 0; k < K; ++k) {
    const double zr = zmode ? om[2 * k] : 0.0, zi = zmode ? om[2 * k + 1] : om[k];
    if (!std::isfinite(zr) || !std::isfinite(zi) || !(zi > 0)) f |= 2;
    for (int i = 0; i < N; ++i) {
      const double re = sg[2 * ((size_t)k * N + i)], im = sg[2 * ((size_t)k * N + i) + 1];
      if (!std::isfinite(re) || !std::isfinite(im)) f |= 4;
      else if (!(zi - im > 0)) f |= 8;
      else if (zi - im < min_im) f |= 16;
    }
  }
  *flag |= f;
}

static std::complex<double> g_of(double mu, double V, double zr, double zi, double sr,
                                 double si) {
  return 1.0 / std::complex<double>(zr + mu - V - sr, zi - si);
}

dyson_status run_solve(dyson_plan* p, Work* w, const Slice* sl, int n, hipStream_t,
                       dyson_report* rep, const std::function<bool()>& abort) {
  int total = 0;
  for (int j = 0; j < n; ++j) total += sl[j].K;
  if (total > w->Kcap || w->plan != p) {
    set_error("batch larger than its workspace");
    return DYSON_EINVAL;
  }
  const int N = p->hp.N;
  for (int j = 0; j < n; ++j) {
    if (abort()) return DYSON_ECANCELLED;  // polled between stages, as between levels
    const Slice& s = sl[j];
    for (int k = 0; k < s.K; ++k) {
      const double zr = s.zmode ? s.omega[2 * k] : 0.0;
      const double zi = s.zmode ? s.omega[2 * k + 1] : s.omega[k];
      for (int i = 0; i < N; ++i) {
        const size_t q = 2 * ((size_t)k * N + i);
        const std::complex<double> g = g_of(p->hp.mu, s.V[i], zr, zi, s.sigma[q], s.sigma[q + 1]);
        s.G[q] = g.real();  // G may be the staging buffer that held Sigma
        s.G[q + 1] = g.imag();
      }
    }
    std::this_thread::sleep_for(std::chrono::microseconds(300));  // overlap the slots
  }
  rep->levels = 1;
  rep->lanczos_steps = total;
  return DYSON_OK;
}
}  // namespace dyson

// ------------------------------------------------------------ the check
static std::atomic<int> fails{0};
#define CHECK(c, ...)                                           \
  do {                                                          \
    if (!(c)) {                                                 \
      std::fprintf(stderr, "FAIL %s:%d ", __FILE__, __LINE__);  \
      std::fprintf(stderr, __VA_ARGS__);                        \
      std::fprintf(stderr, "\n");                               \
      fails.fetch_add(1);                                       \
    }                                                           \
  } while (0)

static dyson_plan* make_plan(dyson_ctx* ctx, int dim, int lx, int ly, int lz, int s) {
  dyson_lattice lat{};
  lat.dim = dim;
  lat.L[0] = lx;
  lat.L[1] = dim > 1 ? ly : 1;
  lat.L[2] = dim > 2 ? lz : 1;
  lat.t = -1.0;
  lat.mu = 0.5;
  dyson_opts o = default_opts();
  o.leaf_edge = s;
  auto* p = new dyson_plan();
  p->ctx = ctx;
  const std::string e = build_plan(lat, o, p->hp);
  if (!e.empty()) {
    std::fprintf(stderr, "plan refused: %s\n", e.c_str());
    std::exit(2);
  }
  return p;
}

struct Job {
  dyson_plan* plan = nullptr;
  int K = 0, mem = DYSON_MEM_HOST, zmode = 0;
  bool cancel = false;
  std::vector<double> V, om, sig, G;
  dyson_req* req = nullptr;
};

static void fill(Job& j, std::mt19937_64& rng) {
  const int N = j.plan->hp.N;
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  j.V.resize(N);
  for (auto& v : j.V) v = 0.1 * u(rng);
  j.om.resize((size_t)j.K * (j.zmode ? 2 : 1));
  for (int k = 0; k < j.K; ++k) {
    if (j.zmode) {
      j.om[2 * k] = u(rng);
      j.om[2 * k + 1] = 0.2 + 0.1 * k;
    } else {
      j.om[k] = 3.14159 * (2 * k + 1) / 20.0;
    }
  }
  j.sig.resize((size_t)j.K * N * 2);
  for (size_t q = 0; q < j.sig.size(); q += 2) {
    j.sig[q] = 0.05 * u(rng);
    j.sig[q + 1] = -0.05 * (1.0 + u(rng));  // Im Sigma < 0: causal
  }
  j.G.assign((size_t)j.K * N * 2, -7.0);
}

static void verify(const Job& j, const char* what) {
  const int N = j.plan->hp.N;
  for (int k = 0; k < j.K; ++k)
    for (int i = 0; i < N; ++i) {
      const size_t q = 2 * ((size_t)k * N + i);
      const double zr = j.zmode ? j.om[2 * k] : 0.0, zi = j.zmode ? j.om[2 * k + 1] : j.om[k];
      const std::complex<double> g =
          1.0 / std::complex<double>(zr + j.plan->hp.mu - j.V[i] - j.sig[q], zi - j.sig[q + 1]);
      if (j.G[q] != g.real() || j.G[q + 1] != g.imag()) {
        CHECK(false, "%s: G differs at k=%d i=%d", what, k, i);
        return;
      }
    }
}

static dyson_status submit(Job& j) {
  return j.zmode ? dyson_submit_z(j.plan, j.K, j.V.data(), j.om.data(), j.sig.data(),
                                  j.G.data(), j.mem, &j.req)
                 : dyson_submit(j.plan, j.K, j.V.data(), j.om.data(), j.sig.data(),
                                j.G.data(), j.mem, &j.req);
}

int main() {
  auto* ctx = new dyson_ctx();
  std::vector<dyson_plan*> plans = {make_plan(ctx, 2, 24, 20, 1, 8), make_plan(ctx, 2, 16, 16, 1, 16),
                                    make_plan(ctx, 3, 8, 6, 7, 4), make_plan(ctx, 1, 40, 1, 1, 8)};
  // a budget of about six frequencies of the largest plan: requests split
  size_t one = 0;
  for (auto* p : plans) one = std::max(one, work_bytes(p, 1));
  ctx->budget = 6 * one;
  CHECK(dyson_serve_config(ctx, 3, 5) == DYSON_OK, "serve_config");

  // several threads submitting concurrently, some requests cancelled
  const int n_threads = 4, per_thread = 12;
  std::vector<std::thread> ths;
  std::atomic<int> done_ok{0}, done_cancelled{0}, batches_multi{0};
  for (int t = 0; t < n_threads; ++t)
    ths.emplace_back([&, t] {
      std::mt19937_64 rng(1000 + t);
      std::vector<Job> jobs(per_thread);
      for (int r = 0; r < per_thread; ++r) {
        Job& j = jobs[r];
        j.plan = plans[(t + r) % plans.size()];
        j.K = 1 + (int)(rng() % 12);
        j.mem = (r % 3 == 0) ? DYSON_MEM_DEVICE : DYSON_MEM_HOST;  // host memory either way here
        j.zmode = (r % 4 == 1);
        j.cancel = (r % 5 == 3);
        fill(j, rng);
        CHECK(submit(j) == DYSON_OK, "submit");
        if (j.cancel) CHECK(dyson_cancel(j.req) == DYSON_OK, "cancel");
        if (r % 6 == 0) {
          int d = 0;
          CHECK(dyson_poll(j.req, &d) == DYSON_OK, "poll");
        }
      }
      for (Job& j : jobs) {
        const dyson_status st = dyson_wait(j.req, -1.0);
        dyson_report rep{};
        CHECK(dyson_req_report(j.req, &rep) == DYSON_OK, "report after wait");
        if (j.cancel) {
          CHECK(st == DYSON_ECANCELLED || st == DYSON_OK, "cancelled request status %d", (int)st);
          if (st == DYSON_OK) verify(j, "request finished before its cancel");
          done_cancelled.fetch_add(1);
        } else {
          CHECK(st == DYSON_OK, "request status %d", (int)st);
          if (st == DYSON_OK) verify(j, "served request");
          if (rep.batches > 1) batches_multi.fetch_add(1);
          done_ok.fetch_add(1);
        }
        CHECK(dyson_release(j.req) == DYSON_OK, "release");
      }
    });
  for (auto& th : ths) th.join();
  CHECK(done_ok.load() + done_cancelled.load() == n_threads * per_thread, "every request ended");
  CHECK(batches_multi.load() > 0, "the budget split some requests into several batches");

  // invalid inputs are refused at submission (both memory modes)
  {
    std::mt19937_64 rng(7);
    for (int mem : {DYSON_MEM_HOST, DYSON_MEM_DEVICE}) {
      Job j;
      j.plan = plans[0];
      j.K = 3;
      j.mem = mem;
      fill(j, rng);
      j.sig[1] = 5.0;  // Im(i w_0 - Sigma) < 0
      CHECK(submit(j) == DYSON_EINVAL, "causality violation refused (mem %d)", mem);
      j.sig[1] = -0.1;
      j.V[3] = std::nan("");
      CHECK(submit(j) == DYSON_EINVAL, "non-finite V refused (mem %d)", mem);
    }
  }

  // a wait with a timeout returns before or at completion, then the request finishes
  {
    std::mt19937_64 rng(9);
    Job j;
    j.plan = plans[0];
    j.K = 12;
    fill(j, rng);
    CHECK(submit(j) == DYSON_OK, "submit (timeout case)");
    const dyson_status st = dyson_wait(j.req, 0.0);
    CHECK(st == DYSON_ETIMEOUT || st == DYSON_OK, "zero timeout status %d", (int)st);
    CHECK(dyson_wait(j.req, -1.0) == DYSON_OK, "wait after timeout");
    verify(j, "request after a timed-out wait");
    CHECK(dyson_release(j.req) == DYSON_OK, "release (timeout case)");
  }

  // several plans in one blocking call (device-mode arrays)
  {
    std::mt19937_64 rng(11);
    std::vector<Job> js(plans.size());
    std::vector<const double*> Vs, oms, sgs;
    std::vector<double*> Gs;
    std::vector<int> Ks;
    for (size_t i = 0; i < plans.size(); ++i) {
      js[i].plan = plans[i];
      js[i].K = 2 + (int)i * 3;
      js[i].mem = DYSON_MEM_DEVICE;
      fill(js[i], rng);
      Vs.push_back(js[i].V.data());
      oms.push_back(js[i].om.data());
      sgs.push_back(js[i].sig.data());
      Gs.push_back(js[i].G.data());
      Ks.push_back(js[i].K);
    }
    std::vector<dyson_report> reps(plans.size());
    CHECK(dyson_solve_batch((int)plans.size(), plans.data(), Ks.data(), Vs.data(), oms.data(),
                            sgs.data(), Gs.data(), nullptr, reps.data()) == DYSON_OK,
          "solve_batch");
    for (auto& j : js) verify(j, "solve_batch");
  }

  for (auto* p : plans) {
    CHECK(p->live_requests.load() == 0, "no live request left on a plan");
    serve_forget_plan(ctx, p);
  }
  delete ctx;  // stops the server: joins the slot threads, frees the workspaces
  for (auto* p : plans) delete p;
  std::printf("served %d requests (%d cancelled), %d split into several batches; %d failures\n",
              done_ok.load() + done_cancelled.load(), done_cancelled.load(), batches_multi.load(),
              fails.load());
  return fails.load() == 0 ? 0 : 1;
}
