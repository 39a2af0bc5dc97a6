// Host driver and C ABI: runs the low-rank correction method level by level,
// all frequencies and all domains of a level as one batch of items.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "../../include/dyson.h"
#include "engine.h"

using namespace dyson;

namespace {

thread_local std::string g_err;

dyson_status fail(dyson_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPC(expr)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(DYSON_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

#define CHECKED(expr)                 \
  do {                                \
    dyson_status s_ = (expr);         \
    if (s_ != DYSON_OK) return s_;    \
  } while (0)

template <typename T>
dyson_status dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(DYSON_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  return DYSON_OK;
}

}  // namespace

namespace dyson {

void set_error(const std::string& msg) { g_err = msg; }
const std::string& get_error() { return g_err; }

hipEvent_t Prof::get() {
  if (used == pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pool.push_back(e);
  }
  return pool[used++];
}
void Prof::reset() {
  used = 0;
  marks.clear();
  for (int c = 0; c < 4; ++c) launches[c] = 0, timed[c] = 0, bytes[c] = 0;
}
Prof::~Prof() {
  for (auto e : pool) (void)hipEventDestroy(e);
}

}  // namespace dyson

namespace {

// Frequencies of one batch: they index the second grid dimension of the
// per-(tile, frequency) launches.
constexpr int kMaxFreqs = 65535;

}  // namespace

namespace dyson {
// Smallest Im H_ii a complex32 (FP16-pair) factorization accepts.  Every
// principal submatrix A of H has Im A >= min_i Im H_ii > 0 (Im H is diagonal
// and positive), so |A^{-1}| <= 1 / min_i Im H_ii bounds the entries of the
// slice inverses; 2^-14 keeps them below 16384, a quarter of the FP16 maximum.
const double kMinImMixed16 = 1.0 / 16384.0;
}  // namespace dyson

namespace {

// Lanczos step cap of a domain with interface size m: the paper allows 5-10
// steps beyond m for m ~ 100; bilinear Lanczos in floating point needs more
// as m grows (m + 11 observed at m = 128), so the allowance scales as m/8.
int step_cap(int m, const dyson_opts& o) {
  if (o.interface_lanczos) return m;  // exactly m steps
  int c = m + std::max(o.extra_steps, (m + 7) / 8);
  if (o.max_rank > 0) c = std::min(c, o.max_rank);
  return c;
}

// Every device buffer of a Work for K frequencies, with its size in bytes.
// The one table serves allocation and the footprint query.
// kq = Lanczos steps the basis must hold; sub = workspace of a concurrent
// level group (it reads the diagonal d and the frequency keys of the main one).
std::vector<std::pair<void**, size_t>> work_table(const dyson_plan* p, Work* w, int K, int kq,
                                                  bool sub) {
  const HostPlan& P = p->hp;
  const size_t NP = (size_t)P.T * P.S;
  const size_t V = (size_t)K * NP * 16;  // bytes per complex vector
  const size_t nq = P.levels.empty() ? 1 : (size_t)(kq + 1);
  const size_t fe = (size_t)K * P.T * P.sy * P.sx * P.sx * 2;  // reals per factor set
  const size_t fsz = (P.opts.precision == DYSON_PREC_MIXED)     ? 4
                     : (P.opts.precision == DYSON_PREC_MIXED16) ? 2
                                                                : 8;
  const size_t ni = (size_t)K * p->nmax;
  // one basis vector: every tile, or (interface form) the tiles holding
  // interface sites only
  const size_t qbytes = P.opts.interface_lanczos && p->nimax > 0  // (no levels: unused)
                            ? (size_t)K * p->nimax * P.S * 16
                            : V;
  std::vector<std::pair<void**, size_t>> t = {
      {(void**)&w->d, V},          {(void**)&w->gacc, V},      {(void**)&w->xB, V},
      {(void**)&w->xH, V},         {(void**)&w->r, V},         {(void**)&w->z, V},
      {(void**)&w->p0, V},         {(void**)&w->p1, V},        {(void**)&w->s, V},
      {(void**)&w->rhs, V},        {(void**)&w->R, V},         {(void**)&w->Dl, V},
      {(void**)&w->Q, qbytes * nq}, {&w->fac[0], fe * fsz},    {&w->fac[1], fe * fsz},
      {(void**)&w->partial, (size_t)K * P.T * 4 * 8},
      {(void**)&w->hpart, (size_t)K * P.T * p->hstride * 16},
      {(void**)&w->h, ni * p->hstride * 16},
      {(void**)&w->cst.done, ni * 4},  {(void**)&w->cst.iters, ni * 4},
      {(void**)&w->cst.bn2, ni * 8},   {(void**)&w->rho2, ni * 32},
      {(void**)&w->alph, ni * 16},
      {(void**)&w->partS, (size_t)K * P.T * 16},
      {(void**)&w->klist, (size_t)K * 4}, {(void**)&w->kalive, (size_t)K * 4},
      {(void**)&w->d_kcount, 16},
      {(void**)&w->lz_stopped, ni * 4}, {(void**)&w->lz_steps, ni * 4},
      {(void**)&w->lz_reorth, ni * 4}, {(void**)&w->lz_armed, ni * 4},
      {(void**)&w->lz_alpha, ni * 16},  {(void**)&w->lz_beta, ni * 16},
      {(void**)&w->lz_unorm2, ni * 8},  {(void**)&w->lz_umax2, ni * 8},
      {(void**)&w->lz_scal, ni * 16},   {(void**)&w->d_count, 16},
      {(void**)&w->d_prof, 64},         {(void**)&w->d_wprof, 4 * ni * 8},
      {(void**)&w->d_fkey, (size_t)K * 8}, {(void**)&w->stage_om, (size_t)K * 16},
      {(void**)&w->d_flag, 16},        {(void**)&w->d_err, 16}};
  if (P.opts.interface_lanczos) {
    // per level: n_nodes items of an mm x mm Hessenberg matrix (mm = the
    // level's largest interface) and the inversion's panels
    size_t hm = 0, pan = 0;
    for (const auto& L : P.levels) {
      size_t mm = 0;
      for (int m : L.m) mm = std::max<size_t>(mm, (size_t)m);
      hm = std::max(hm, (size_t)L.n_nodes * mm * mm);
      pan = std::max(pan, (size_t)L.n_nodes * mm * 32);
    }
    t.push_back({(void**)&w->Vb, V * nq});
    t.push_back({(void**)&w->Hm, (size_t)K * hm * 16});
    t.push_back({(void**)&w->gjC, (size_t)K * pan * 16});
    t.push_back({(void**)&w->gjR, (size_t)K * pan * 16});
    t.push_back({(void**)&w->gjQ, ni * 32 * 32 * 16});
    t.push_back({(void**)&w->f1mask, ni * 4});
  }
  if (sub) {
    std::vector<std::pair<void**, size_t>> keep;
    for (auto& e : t)
      if (e.first != (void**)&w->d && e.first != (void**)&w->d_fkey &&
          e.first != (void**)&w->stage_om && e.first != (void**)&w->d_flag &&
          e.first != (void**)&w->d_err)
        keep.push_back(e);
    return keep;
  }
  // mixed plans keep complex128 leaf factors beside the low-precision ones;
  // FP64 plans use the first factor slot for them
  if (P.opts.precision != DYSON_PREC_FP64) t.push_back({(void**)&w->fac64, fe * 8});
  return t;
}

size_t table_bytes(const std::vector<std::pair<void**, size_t>>& t) {
  size_t b = 0;
  for (auto& e : t) b += (e.second + 255) / 256 * 256;
  return b;
}

void* dev_alloc(const dyson_ctx* c, size_t n, hipStream_t s) {
  if (c->has_alloc) return c->alloc.alloc(n, (void*)s, c->alloc.user);
  void* ptr = nullptr;
  if (hipMalloc(&ptr, n) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return ptr;
}

void dev_free(const dyson_ctx* c, void* ptr, hipStream_t s) {
  if (!ptr) return;
  if (c->has_alloc) c->alloc.free(ptr, (void*)s, c->alloc.user);
  else (void)hipFree(ptr);
}

}  // namespace

namespace dyson {

void* ctx_alloc(const dyson_ctx* c, size_t bytes, hipStream_t s) { return dev_alloc(c, bytes, s); }
void ctx_free(const dyson_ctx* c, void* ptr, hipStream_t s) { dev_free(c, ptr, s); }

std::vector<std::vector<int>> level_groups(const dyson_plan* p) {
  const HostPlan& P = p->hp;
  const int L = (int)P.levels.size();
  const int C = std::max(1, std::min(P.opts.level_streams, L));
  std::vector<std::vector<int>> g(C);
  if (C == 1) {
    for (int l = L - 1; l >= 0; --l) g[0].push_back(l);
    return g;
  }
  // longest processing time first on the sequential Lanczos step count
  std::vector<int> wt(L), order(L);
  for (int l = 0; l < L; ++l) {
    int mx = 0;
    for (int m : P.levels[l].m) mx = std::max(mx, m);
    wt[l] = step_cap(mx, P.opts);
    order[l] = l;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return wt[a] > wt[b]; });
  std::vector<long long> load(C, 0);
  for (int l : order) {
    int best = 0;
    for (int c = 1; c < C; ++c)
      if (load[c] < load[best]) best = c;
    g[best].push_back(l);
    load[best] += wt[l];
  }
  for (auto& v : g) std::sort(v.begin(), v.end(), std::greater<int>());  // bottom-up
  return g;
}

namespace {

// Lanczos steps a group's basis must hold.
int group_kq(const dyson_plan* p, const std::vector<int>& levels) {
  int kq = 1;
  for (int l : levels)
    for (int m : p->hp.levels[l].m) kq = std::max(kq, step_cap(m, p->hp.opts) + 1);
  return kq;
}

}  // namespace

size_t work_bytes(const dyson_plan* p, int K) {
  Work tmp;
  size_t b = table_bytes(work_table(p, &tmp, K, p->kcap, false));
  const auto g = level_groups(p);
  for (size_t c = 1; c < g.size(); ++c)
    b += table_bytes(work_table(p, &tmp, K, group_kq(p, g[c]), true));
  return b;
}

size_t carved_bytes(const dyson_plan* p, int K) {
  Work tmp;
  return table_bytes(work_table(p, &tmp, K, p->kcap, false));
}

dyson_status carve_work(const dyson_plan* p, Work* w, int K, char* base, size_t cap) {
  const size_t need = carved_bytes(p, K);
  if (need > cap)
    return fail(DYSON_EINVAL, "the allocation-free solve of " + std::to_string(K) +
                                  " frequencies on this plan needs " + std::to_string(need) +
                                  " bytes of scratch; the maximum is " + std::to_string(cap));
  w->plan = p;
  w->carved = true;
  size_t off = 0;
  for (auto& e : work_table(p, w, K, p->kcap, false)) {
    *e.first = base + off;
    off += (e.second + 255) / 256 * 256;
  }
  if (p->hp.opts.precision == DYSON_PREC_FP64) w->fac64 = (double*)w->fac[0];
  w->h_count = w->h_static;
  w->Kcap = K;
  w->kq = p->kcap;
  w->bytes = off;
  w->fac_g[0] = w->fac_g[1] = -1000;
  return DYSON_OK;
}

void free_work(Work* w, hipStream_t s) {
  if (w->carved) {  // slices of a region the Work does not own
    *w = Work{};
    return;
  }
  const dyson_ctx* c = w->plan ? w->plan->ctx : nullptr;
  if (c) (void)hipSetDevice(c->device);
  for (size_t i = 0; i < w->sub.size(); ++i) {
    if (w->sub[i]) free_work(w->sub[i].get(), w->sub_stream[i]);
    if (w->sub_stream[i]) (void)hipStreamDestroy(w->sub_stream[i]);
  }
  w->sub.clear();
  w->sub_stream.clear();
  if (w->ev) (void)hipEventDestroy(w->ev);
  w->ev = nullptr;
  if (c)
    for (void* a : w->allocs) dev_free(c, a, s);
  w->allocs.clear();
  if (w->h_count) (void)hipHostFree(w->h_count);
  w->h_count = nullptr;
  w->Kcap = 0;
  w->bytes = 0;
  w->plan = nullptr;
  w->fac_g[0] = w->fac_g[1] = -1000;
  w->pred.clear();
  for (auto& g : w->graphs) (void)hipGraphExecDestroy(g.second);
  w->graphs.clear();
  w->graphs_broken = false;
}

namespace {

dyson_status alloc_table(const dyson_plan* p, Work* w, int K, int kq, bool sub, hipStream_t s) {
  w->plan = p;
  for (auto& e : work_table(p, w, K, kq, sub)) {
    void* ptr = dev_alloc(p->ctx, e.second ? e.second : 1, s);
    if (!ptr) return fail(DYSON_ENOMEM, "device allocation of " + std::to_string(e.second) +
                                            " bytes failed");
    *e.first = ptr;
    w->allocs.push_back(ptr);
    w->bytes += (e.second + 255) / 256 * 256;
  }
  if (p->hp.opts.precision == DYSON_PREC_FP64 && !sub) w->fac64 = (double*)w->fac[0];
  launch_zero(w->d_wprof, 4 * (size_t)K * p->nmax * sizeof(unsigned long long), s);
  if (hipHostMalloc((void**)&w->h_count, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    w->h_count = nullptr;
    return fail(DYSON_ENOMEM, "pinned host allocation failed");
  }
  w->Kcap = K;
  w->kq = kq;
  return DYSON_OK;
}

}  // namespace

dyson_status ensure_work(const dyson_plan* p, Work* w, int K, hipStream_t s) {
  if (w->plan == p && K <= w->Kcap) return DYSON_OK;
  if (w->carved) return fail(DYSON_EINVAL, "scratch workspace is smaller than the call");
  HIPC(hipSetDevice(p->ctx->device));
  free_work(w, s);
  dyson_status st = alloc_table(p, w, K, p->kcap, false, s);
  const auto g = level_groups(p);
  if (st == DYSON_OK && g.size() > 1) {
    if (hipEventCreateWithFlags(&w->ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      w->ev = nullptr;
      st = fail(DYSON_EDEVICE, "hipEventCreate failed");
    }
    for (size_t c = 1; c < g.size() && st == DYSON_OK; ++c) {
      w->sub.push_back(std::make_unique<Work>());
      w->sub_stream.push_back(nullptr);
      if (hipStreamCreateWithFlags(&w->sub_stream.back(), hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        w->sub_stream.back() = nullptr;
        st = fail(DYSON_EDEVICE, "hipStreamCreate failed");
        break;
      }
      Work* sw = w->sub.back().get();
      st = alloc_table(p, sw, K, group_kq(p, g[c]), true, w->sub_stream.back());
      w->bytes += sw->bytes;
    }
  }
  if (st != DYSON_OK) {
    const std::string msg = g_err;
    free_work(w, s);
    g_err = msg;
    return st;
  }
  return DYSON_OK;
}

}  // namespace dyson

namespace {

// ----------------------------------------------------------- the solver
struct Run {
  dyson_plan* p;
  Work* w;
  int K;
  hipStream_t s;
  const HostPlan& P() const { return p->hp; }

  // Time a launch when profiling, class c.  profile = 1: the inner-solve
  // update kernel only (the dominant kernel); profile >= 2: every class.
  // Events around every launch cost about 4% of a solve, so a fixed
  // pseudo-random one in sixteen of a class's launches is timed (Knuth's
  // multiplicative hash of the launch index) and the report scales the sample
  // to all launches; the algorithmic bytes are counted for every launch.
  template <typename Fn>
  void timed(int c, Fn fn) {
    Prof& pr = w->prof;
    if (!pr.on) {
      fn();
      return;
    }
    const unsigned long long n = (unsigned long long)pr.launches[c]++;
    const bool sample = (P().opts.profile >= 2 || c == 0) &&
                        ((uint32_t)(n * 2654435761ull) >> 28) == 0;
    if (!sample) {
      fn();
      return;
    }
    hipEvent_t a = pr.get(), b = pr.get();
    (void)hipEventRecord(a, s);
    fn();
    (void)hipEventRecord(b, s);
    pr.marks.push_back({c, {a, b}});
    pr.timed[c] += 1;
  }

  dyson_status count_open(const int* flags, int n, int* out) {
    launch_count_open(flags, n, w->d_count, s);
    HIPC(hipMemcpyAsync(w->h_count, w->d_count, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    *out = w->h_count[0];
    return DYSON_OK;
  }

  // Factor the tile blocks of graph g (cached in one of two slots).
  dyson_status factors_for(int g, int level, void** fac) {
    for (int i = 0; i < 2; ++i)
      if (w->fac_g[i] == g) {
        *fac = w->fac[i];
        return DYSON_OK;
      }
    // evict the slot not holding the other graph of this level
    int slot = (w->fac_g[0] == g + 1 || w->fac_g[0] == g - 1) ? 1 : 0;
    (void)level;  // every tile is factored: a graph is shared by two levels
    launch_factor(p->geom, K, g, nullptr, w->d, w->fac[slot],
                  P().opts.precision == DYSON_PREC_MIXED, P().opts.precision == DYSON_PREC_MIXED16,
                  s);
    HIPC(hipGetLastError());
    w->fac_g[slot] = g;
    *fac = w->fac[slot];
    return DYSON_OK;
  }

  // COCG on graph g for every item of `level`, x = A_g^{-1} b.  Two launches
  // per iteration; the host polls the device's open-item count only near the
  // iteration count the previous solve of the same kind needed.
  // Iterations [it0, it0 + n) of an inner solve: stencil and update per
  // iteration (p_old and p_new trade places), and after every fourth stencil
  // the open-frequency compaction (in between, the list is a superset of the
  // open frequencies, which only costs the closed units a quick exit).
  void launch_iterations(CocgLaunch c, int it0, int n) {
    for (int i = 0; i < n; ++i) {
      timed(1, [&] { launch_cocg_stencil(c, it0 + i, s); });
      if (((it0 + i) & 3) == 3)
        launch_cocg_compact(c, it0 + i + 2, w->klist, w->d_kcount, s);
      timed(0, [&] { launch_cocg_update(c, it0 + i, s); });
      std::swap(c.p_old, c.p_new);
    }
  }

  // The same iterations as one captured HIP graph, made on first use and
  // replayed for every later solve with the same launch arguments (the
  // buffers of a Work do not move between calls).  false: not available
  // (the caller launches directly).
  bool replay_iterations(const CocgLaunch& c, int it0, int n) {
    if (w->graphs_broken) return false;
    std::string key(reinterpret_cast<const char*>(&c), sizeof(c));
    key.append(reinterpret_cast<const char*>(&it0), sizeof(it0));
    key.append(reinterpret_cast<const char*>(&n), sizeof(n));
    auto f = w->graphs.find(key);
    if (f == w->graphs.end()) {
      if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        w->graphs_broken = true;
        return false;
      }
      launch_iterations(c, it0, n);
      hipGraph_t gr = nullptr;
      hipGraphExec_t ge = nullptr;
      const bool ok = hipStreamEndCapture(s, &gr) == hipSuccess && gr &&
                      hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0) == hipSuccess;
      if (gr) (void)hipGraphDestroy(gr);
      if (!ok) {
        (void)hipGetLastError();
        w->graphs_broken = true;
        return false;
      }
      f = w->graphs.emplace(std::move(key), ge).first;
    }
    return hipGraphLaunch(f->second, s) == hipSuccess;
  }

  dyson_status cocg(int level, int g, const void* fac, const double* b, double* x,
                    bool skip_stopped = true) {
    const DevLevel& L = p->lv[level];
    const HostPlan& HP = P();
    CocgLaunch c;
    std::memset(&c, 0, sizeof(c));  // padding included: the struct keys the graph cache
    c.G = p->geom;
    c.K = K;
    c.g = g;
    c.tile_node = L.tile_node;
    c.n_nodes = L.n;
    c.item_skip = skip_stopped ? w->lz_stopped : nullptr;
    c.st = w->cst;
    c.d = w->d;
    c.x = x;
    c.r = w->r;
    c.z = w->z;
    c.p_old = w->p0;
    c.p_new = w->p1;
    c.s = w->s;
    c.fac = fac;
    c.fp32 = HP.opts.precision == DYSON_PREC_MIXED;
    c.fp16 = HP.opts.precision == DYSON_PREC_MIXED16;
    c.wctr = w->prof.on ? w->d_wprof : nullptr;
    c.tlo = L.tlo;
    c.thi = L.thi;
    c.n_items = K * L.n;
    c.partS = w->partS;
    c.partU = w->partial;
    c.rho2 = w->rho2;
    c.alph = w->alph;
    c.tol2 = HP.opts.inner_tol * HP.opts.inner_tol;
    const int slot = 2 * level + (g == level ? 0 : 1);
    if ((int)w->pred.size() <= slot) w->pred.resize(slot + 1, 0);
    // the stencil and update launches run over the frequencies that still
    // have an open item (stamped by the check and the stencil, compacted
    // after each)
    c.kalive = w->kalive;
    launch_zero(w->kalive, (size_t)K * sizeof(int), s);
    launch_cocg_init(c, b, s);
    launch_cocg_check(c, 0, w->d_count, s);
    launch_cocg_compact(c, 1, w->klist, w->d_kcount, s);
    c.klist = w->klist;
    c.kcount = w->d_kcount;
    const int maxit = HP.opts.max_inner_iters;
    int it = 0, open = 1;
    int check_at = std::max(1, w->pred[slot] - 1);
    // iterations before the first poll go in chunks of kChunk (an even
    // count: p_old and p_new end where they started) as captured graphs
    constexpr int kChunk = 8;
    const bool graphs = HP.opts.inner_graphs >= 0 && !w->prof.on && !w->carved;
    while (it < maxit) {
      const int stop = std::min(check_at, maxit);
      if (graphs && it + kChunk <= stop && replay_iterations(c, it, kChunk)) {
        it += kChunk;
      } else {
        launch_iterations(c, it, 1);
        std::swap(c.p_old, c.p_new);
        ++it;
      }
      if (it >= check_at || it == maxit) {
        launch_cocg_check(c, it, w->d_count, s);
        HIPC(hipMemcpyAsync(w->h_count, w->d_count, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        open = w->h_count[0];
        if (open == 0) break;
        check_at = it + (it < 8 ? 1 : 2);
      }
    }
    // closes the items still open: applies the x update deferred from an even
    // last iteration (also to items stopped by max_inner_iters)
    c.flush = 1;
    if (it > 0) launch_cocg_stencil(c, it, s);
    HIPC(hipGetLastError());
    if (open != 0) {
      w->pending = DYSON_ENOCONV;
      g_err = "inner COCG solve hit max_inner_iters";
    }
    if (w->prof.on) launch_prof_collect(w->d_wprof, K * L.n, 2, 0, w->d_prof, s);
    w->pred[slot] = it;
    w->stat_inner += it;
    w->stat_inner_max = std::max(w->stat_inner_max, it);
    return DYSON_OK;
  }

  LzArgs lz_args(int level) {
    LzArgs a{};
    a.G = p->geom;
    a.level = level;
    a.tile_node = p->lv[level].tile_node;
    a.n_nodes = p->lv[level].n;
    a.seed = P().opts.seed;
    a.fkey = w->d_fkey;
    a.stopped = w->lz_stopped;
    a.steps = w->lz_steps;
    a.alpha = w->lz_alpha;
    a.beta = w->lz_beta;
    a.unorm2 = w->lz_unorm2;
    a.umax2 = w->lz_umax2;
    a.scal = w->lz_scal;
    a.partial = w->partial;
    a.hpart = w->hpart;
    a.h = w->h;
    a.hstride = p->hstride;
    a.tlo = p->lv[level].tlo;
    a.thi = p->lv[level].thi;
    a.n_items = K * p->lv[level].n;
    a.wctr = w->prof.on ? w->d_wprof + 2 * (size_t)K * p->nmax : nullptr;
    a.reorth = w->lz_reorth;
    a.armed = w->lz_armed;
    return a;
  }

  dyson_status reset_items(int level) {
    const size_t ni = (size_t)K * p->lv[level].n;
    launch_zero(w->lz_stopped, ni * sizeof(int), s);
    launch_zero(w->lz_steps, ni * sizeof(int), s);
    launch_zero(w->lz_beta, ni * 2 * sizeof(double), s);
    return DYSON_OK;
  }

  // u = X_level q for every item (eqs. (10)-(12), solve of (10) started at w).
  dyson_status xmatvec(int level, const double* q, double* u) {
    void *facB = nullptr, *facH = nullptr;
    CHECKED(factors_for(level + 1, level, &facB));
    CHECKED(cocg(level, level + 1, facB, q, w->xB));        // w = B^{-1} q_B   (11)
    LzArgs a = lz_args(level);
    launch_lz_defect(a, K, q, w->xB, w->rhs, s);             // q - H w
    CHECKED(factors_for(level, level, &facH));
    CHECKED(cocg(level, level, facH, w->rhs, u));            // u = v - w        (10),(12)
    return DYSON_OK;
  }

  // Full re-orthogonalization of r against the basis: classical Gram-Schmidt,
  // repeated for the items whose first pass removed most of r (|r'| <
  // |r| / sqrt 2), which keeps the basis orthogonal to working precision.
  // after_reduce(pass) runs once the pass's coefficients are in a.h; D (the
  // streamed diagonal of the X form) may be null.
  // eta2 > 1 makes the second pass unconditional.
  template <typename Hook>
  void cgs2(const LzArgs& a, const DevLevel& L, int nvec, double* D, Hook after_reduce,
            double eta2 = 0.5) {
    (void)L;
    // doubles between consecutive basis vectors (compact storage: the listed tiles)
    const size_t qstride =
        (size_t)K * (a.qcompact ? (size_t)a.n_tlist : (size_t)P().T) * P().S * 2;
    for (int pass = 0; pass < 2; ++pass) {
      timed(3, [&] { launch_cgs_dot(a, K, w->Q, qstride, nvec, w->R, pass, s); });
      launch_cgs_reduce(a, K, a.tlo, a.thi, nvec, pass, s);
      after_reduce(pass);
      timed(2, [&] { launch_cgs_update(a, K, w->Q, qstride, nvec, w->R, D, pass, s); });
      if (pass == 0) launch_cgs_decide(a, K, a.tlo, a.thi, nvec, eta2, s);
    }
  }
  void cgs2(const LzArgs& a, const DevLevel& L, int nvec) {
    cgs2(a, L, nvec, w->Dl, [](int) {});
  }

  // One correction level in the interface form: bilinear Lanczos on the
  // Schur complement S of every (domain, frequency) for exactly m steps
  // (S p = (H (p - B^{-1} E p))|_C: one inner solve per step), the projected
  // Hessenberg matrix H accumulated per item, then H^{-1} for every item at
  // once and diag(X) = diag(V H^{-1} V^T) added to the running diagonal.  An
  // item whose bilinear form breaks down (or whose residual vanishes before
  // m steps) is redone from a fresh start vector, at most twice.
  dyson_status lanczos_level_iface(int level, std::vector<int>* steps_out) {
    const DevLevel& L = p->lv[level];
    const HostPlan& HP = P();
    const size_t V = (size_t)K * HP.T * HP.S * 2;
    LzArgs a = lz_args(level);
    a.iface = 1;
    // the basis lives on the interface tiles only, stored compactly (every
    // correction level has interface sites, so the list is never empty)
    if (L.n_itiles <= 0) return fail(DYSON_EINVAL, "correction level without interface sites");
    a.tlist = L.itiles;
    a.n_tlist = L.n_itiles;
    a.tlo = L.ilo;
    a.thi = L.ihi;
    a.qcompact = 1;
    a.tpos = L.itpos;
    const size_t Vq = (size_t)K * (a.qcompact ? (size_t)a.n_tlist : (size_t)HP.T) * HP.S * 2;
    auto Qj = [&](int j) { return w->Q + (size_t)j * Vq; };
    auto Vj = [&](int j) { return w->Vb + (size_t)j * V; };
    CHECKED(reset_items(level));
    launch_zero(w->Dl, V * sizeof(double), s);
    const int n_items = K * L.n;
    int mm = 0;
    for (int m : HP.levels[level].m) mm = std::max(mm, m);
    launch_zero(w->Hm, (size_t)n_items * mm * mm * 16, s);
    double brk = HP.opts.breakdown_tol;
    std::vector<int> st(n_items), stop(n_items);
    void* facB = nullptr;
    for (int attempt = 0; attempt < 3; ++attempt) {
      if (attempt > 0) launch_f1_hzero(a, w->Hm, mm, s);
      launch_lz_random(a, K, Qj(0), (uint64_t)attempt, s);
      launch_lz_scalars(a, K, a.tlo, a.thi, L.m, 0, 0, HP.opts.lanczos_tol, brk, 0, s);
      launch_lz_scale(a, K, Qj(0), s);
      HIPC(hipGetLastError());
      for (int j = 0; j < mm; ++j) {
        int open = 0;
        CHECKED(count_open(w->lz_stopped, n_items, &open));
        if (open == 0) break;
        const double* q = Qj(j);
        launch_f1_rhs(a, K, q, w->rhs, s);                       // E p
        CHECKED(factors_for(level + 1, level, &facB));
        CHECKED(cocg(level, level + 1, facB, w->rhs, w->xB));    // u = B^{-1} E p
        if (w->pending != DYSON_OK) break;
        launch_f1_smat(a, K, w->d, q, w->xB, w->xH, Vj(j), s);   // S p, v = p + u
        launch_lz_alpha(a, K, q, w->xH, s);
        launch_lz_scalars(a, K, a.tlo, a.thi, L.m, 1, j, HP.opts.lanczos_tol, brk, 0, s);
        launch_lz_recur(a, K, q, j > 0 ? Qj(j - 1) : nullptr, w->xH, w->R, nullptr, s);
        cgs2(a, L, j + 1, nullptr, [&](int pass) { launch_f1_hcol(a, w->Hm, mm, j, pass, s); });
        launch_lz_norms(a, K, w->R, s);
        const int force = (HP.opts.fault_step == j + 1 && attempt < HP.opts.fault_attempts);
        launch_lz_scalars(a, K, a.tlo, a.thi, L.m, 2, j, HP.opts.lanczos_tol, brk, force, s);
        launch_f1_hcol(a, w->Hm, mm, j, 2, s);
        if (j + 1 < w->kq) launch_lz_next(a, K, w->R, Qj(j + 1), s);
        HIPC(hipGetLastError());
        // items whose basis met an invariant subspace go on from a fresh
        // real random direction, orthogonalized against the basis in two
        // full passes (a random vector is not close to the basis, so the
        // selective test's premise does not hold for it)
        launch_f1_mask(a, w->f1mask, s);
        int fresh = 0;
        CHECKED(count_open(w->f1mask, n_items, &fresh));
        if (fresh > 0 && j + 1 < w->kq) {
          LzArgs b = a;
          b.stopped = w->f1mask;
          launch_lz_random(b, K, w->R, (uint64_t)(1000 + attempt) * 1000003ull + (uint64_t)j, s, 1);
          cgs2(b, L, j + 1, nullptr, [](int) {}, 1e300);
          launch_lz_norms(b, K, w->R, s);
          launch_lz_scalars(b, K, a.tlo, a.thi, L.m, 3, j, HP.opts.lanczos_tol, brk, 0, s);
          launch_lz_next(b, K, w->R, Qj(j + 1), s);
          w->stat_restarts += fresh;
        }
        launch_f1_settle(a, s);
        HIPC(hipGetLastError());
      }
      HIPC(hipMemcpyAsync(stop.data(), w->lz_stopped, n_items * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPC(hipMemcpyAsync(st.data(), w->lz_steps, n_items * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      int bad = 0;
      for (int i = 0; i < n_items; ++i) bad += (stop[i] == 3);
      if (bad == 0 || w->pending != DYSON_OK) break;
      if (attempt == 2) {
        w->pending = DYSON_EBREAKDOWN;
        g_err = "Lanczos breakdown persisted after restarts";
        break;
      }
      w->stat_restarts += bad;
      brk *= 1e-2;
      launch_lz_reopen(a, K, w->Dl, s);
      HIPC(hipGetLastError());
    }
    if (w->prof.on) launch_prof_collect(a.wctr, n_items, 2, 2, w->d_prof, s);
    if (w->pending == DYSON_OK) {
      launch_f1_hpad(a, w->Hm, mm, s);
      launch_gj_invert(w->Hm, mm, n_items, w->gjC, w->gjR, w->gjQ, s);
      launch_f1_diag(a, K, w->Vb, V, w->Hm, mm, w->Dl, s);
      launch_add_into(a, K, w->Dl, w->gacc, s);
      HIPC(hipGetLastError());
    }
    if (steps_out) *steps_out = st;
    return DYSON_OK;
  }

  // One correction level: bilinear Lanczos on X for every (domain, frequency),
  // diag(Q H Q^T) gathered in Dl and added to the running diagonal at the end.
  // An item whose bilinear form breaks down is redone from a fresh start
  // vector (its partial diagonal is discarded), at most twice.
  dyson_status lanczos_level(int level, std::vector<int>* steps_out) {
    const DevLevel& L = p->lv[level];
    const HostPlan& HP = P();
    const size_t V = (size_t)K * HP.T * HP.S * 2;
    auto Qj = [&](int j) { return w->Q + (size_t)j * V; };
    CHECKED(reset_items(level));
    launch_zero(w->Dl, V * sizeof(double), s);
    LzArgs a = lz_args(level);
    const int n_items = K * L.n;
    // |r^T r| <= brk |r|^2: redo the item; each further attempt accepts a
    // 100x smaller ratio, so a strict threshold buys accuracy on the first
    // attempt without failing an item whose fresh starts all come close
    double brk = HP.opts.breakdown_tol;
    int kmax = 0;
    for (int m : HP.levels[level].m) kmax = std::max(kmax, step_cap(m, HP.opts));
    kmax = std::min(kmax, w->kq);
    std::vector<int> st(n_items), stop(n_items);
    for (int attempt = 0; attempt < 3; ++attempt) {
      // start vector, normalized in the bilinear "norm"
      launch_lz_random(a, K, Qj(0), (uint64_t)attempt, s);
      launch_lz_scalars(a, K, L.tlo, L.thi, L.mcap, 0, 0, HP.opts.lanczos_tol, brk, 0, s);
      launch_lz_scale(a, K, Qj(0), s);
      HIPC(hipGetLastError());
      const bool verbose = std::getenv("DYSON_VERBOSE") != nullptr;
      for (int j = 0; j < kmax; ++j) {
        int open = 0;
        CHECKED(count_open(w->lz_stopped, n_items, &open));
        if (open == 0) break;
        if (verbose && j > 0 && j % 256 == 0) {
          std::fprintf(stderr, "[dyson] level %d step %d: %d of %d items open\n", level, j, open,
                       n_items);
          std::fflush(stderr);
        }
        const double* q = Qj(j);
        CHECKED(xmatvec(level, q, w->xH));
        if (w->pending != DYSON_OK) break;  // an inner solve failed: the level cannot finish
        launch_lz_alpha(a, K, q, w->xH, s);
        launch_lz_scalars(a, K, L.tlo, L.thi, L.mcap, 1, j, HP.opts.lanczos_tol, brk, 0, s);
        launch_lz_recur(a, K, q, j > 0 ? Qj(j - 1) : nullptr, w->xH, w->R, w->Dl, s);
        cgs2(a, L, j + 1);
        launch_lz_norms(a, K, w->R, s);
        const int force = (HP.opts.fault_step == j + 1 && attempt < HP.opts.fault_attempts);
        launch_lz_scalars(a, K, L.tlo, L.thi, L.mcap, 2, j, HP.opts.lanczos_tol, brk, force, s);
        if (j + 1 < w->kq) launch_lz_next(a, K, w->R, Qj(j + 1), s);
        HIPC(hipGetLastError());
      }
      HIPC(hipMemcpyAsync(stop.data(), w->lz_stopped, n_items * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPC(hipMemcpyAsync(st.data(), w->lz_steps, n_items * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      int bad = 0;
      for (int i = 0; i < n_items; ++i) {
        bad += (stop[i] == 3);
        if (stop[i] == 2) w->stat_capped += 1;
      }
      if (std::getenv("DYSON_VERBOSE")) {
        int hist[5] = {0, 0, 0, 0, 0};
        for (int i = 0; i < n_items; ++i) hist[std::min(std::max(stop[i], 0), 4)]++;
        std::fprintf(stderr, "[dyson] level %d attempt %d: stop codes open=%d exhausted=%d cap=%d breakdown=%d\n",
                     level, attempt, hist[0], hist[1], hist[2], hist[3]);
      }
      if (bad == 0 || w->pending != DYSON_OK) break;
      if (attempt == 2) {
        w->pending = DYSON_EBREAKDOWN;
        g_err = "Lanczos breakdown persisted after restarts";
        break;
      }
      w->stat_restarts += bad;
      brk *= 1e-2;
      launch_lz_reopen(a, K, w->Dl, s);
      HIPC(hipGetLastError());
    }
    if (w->prof.on) launch_prof_collect(a.wctr, n_items, 2, 2, w->d_prof, s);
    launch_add_into(a, K, w->Dl, w->gacc, s);
    HIPC(hipGetLastError());
    if (steps_out) *steps_out = st;
    return DYSON_OK;
  }
};

// Clears the per-call statistics and the factor cache of a Work.
dyson_status begin_call(dyson_plan* p, Work* w, int K, hipStream_t s) {
  if (!p || !p->ctx) return fail(DYSON_EINVAL, "plan has no device context");
  if (K < 1 || K > kMaxFreqs) return fail(DYSON_EINVAL, "K must be in [1, 65535]");
  HIPC(hipSetDevice(p->ctx->device));
  CHECKED(ensure_work(p, w, K, s));
  w->pending = DYSON_OK;
  w->stat_inner = 0;
  w->stat_inner_max = 0;
  w->stat_restarts = 0;
  w->stat_capped = 0;
  w->fac_g[0] = w->fac_g[1] = -1000;  // factors depend on d, which changes per call
  launch_freq_keys(nullptr, 0, K, w->d_fkey, s);
  return DYSON_OK;
}

}  // namespace

namespace dyson {

dyson_status validate_slices(const dyson_plan* p, Work* w, const Slice* sl, int n, hipStream_t s) {
  const int N = p->hp.N;
  launch_zero(w->d_flag, sizeof(int), s);
  for (int j = 0; j < n; ++j) {
    if (sl[j].K < 1) return fail(DYSON_EINVAL, "K must be >= 1");
    if (!sl[j].V || !sl[j].omega || !sl[j].sigma || !sl[j].G)
      return fail(DYSON_EINVAL, "null input or output pointer");
    launch_validate(N, sl[j].K, sl[j].V, sl[j].omega, sl[j].zmode, sl[j].sigma,
                    p->hp.opts.precision == DYSON_PREC_MIXED16 ? kMinImMixed16 : 0.0, w->d_flag, s);
  }
  HIPC(hipGetLastError());
  HIPC(hipMemcpyAsync(w->h_count, w->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  const int f = w->h_count[0];
  if (f & 1) return fail(DYSON_EINVAL, "V contains a non-finite value");
  if (f & 2) return fail(DYSON_EINVAL, "frequencies must be finite with w_k > 0 (Im z_k > 0)");
  if (f & 4) return fail(DYSON_EINVAL, "Sigma contains a non-finite value");
  if (f & 8) return fail(DYSON_EINVAL, "Im(z_k - Sigma_i) must be > 0 (causal self-energy)");
  if (f & 16)
    return fail(DYSON_EUNSUPPORTED,
                "DYSON_PREC_MIXED16 needs Im(z_k - Sigma_i) >= 2^-14: its FP16 factor entries "
                "reach 1 / min Im H_ii; use DYSON_PREC_MIXED or DYSON_PREC_FP64");
  return DYSON_OK;
}

dyson_status run_solve(dyson_plan* p, Work* w, const Slice* sl, int n, hipStream_t s,
                       dyson_report* rep, const std::function<bool()>& abort) {
  auto t0 = std::chrono::steady_clock::now();
  int K = 0;
  for (int j = 0; j < n; ++j) K += sl[j].K;
  CHECKED(begin_call(p, w, K, s));
  const HostPlan& P = p->hp;
  w->prof.reset();
  w->prof.on = P.opts.profile != 0 && !w->carved;
  if (w->prof.on) launch_zero(w->d_prof, 8 * sizeof(unsigned long long), s);
  Run run{p, w, K, s};
  const size_t NP = (size_t)P.T * P.S;
  // a1: diagonal of H, each slice into its rows of the batch
  for (int j = 0, k0 = 0; j < n; k0 += sl[j].K, ++j) {
    launch_freq_keys(sl[j].omega, sl[j].zmode, sl[j].K, w->d_fkey + k0, s);
    launch_assemble(p->geom, sl[j].K, P.mu, sl[j].V, sl[j].omega, sl[j].zmode, sl[j].sigma,
                    w->d + (size_t)k0 * NP * 2, s);
  }
  // a3/a4: leaf factorization and diag(B^{-1})
  const size_t V = (size_t)K * NP * 2;
  launch_zero(w->gacc, V * sizeof(double), s);
  // FP64 plans keep the leaf factors (FP64 buffers); mixed plans only take the
  // diagonal here and factor the preconditioner again in complex64
  const bool keep = P.opts.precision == DYSON_PREC_FP64;
  launch_factor_diag(p->geom, K, w->d, w->fac64, w->gacc, s);
  HIPC(hipGetLastError());
  if (keep && !P.levels.empty()) {
    // the leaf factors double as the preconditioner of the deepest B graph
    w->fac_g[0] = (int)P.levels.size();
  }
  // a5-a9: the corrections.  Each level adds its own diag(X_l); the levels
  // of a group run bottom-up, the groups concurrently on their own streams.
  std::vector<std::vector<int>> groups = level_groups(p);
  if (w->carved) {  // one group, bottom-up, on the call's stream
    groups.assign(1, {});
    for (int l = (int)P.levels.size() - 1; l >= 0; --l) groups[0].push_back(l);
  }
  const int G = (int)groups.size();
  std::vector<dyson_status> gst(G, DYSON_OK);
  std::vector<std::string> gerr(G);
  std::vector<std::vector<int>> lsteps_of(P.levels.size());
  const bool verbose = std::getenv("DYSON_VERBOSE") != nullptr;
  if (G > 1) {
    // d, keys and leaf results are ready: every group's stream waits on the
    // event here, before any group starts (a group may capture graphs on its
    // stream, and a wait on an event recorded on a capturing stream fails)
    HIPC(hipEventRecord(w->ev, s));
    for (int g = 1; g < G; ++g)
      if (hipStreamWaitEvent(w->sub_stream[g - 1], w->ev, 0) != hipSuccess)
        return fail(DYSON_EDEVICE, "level group set-up failed");
  }
  auto run_group = [&](int g) {
    Work* gw = (g == 0) ? w : w->sub[g - 1].get();
    hipStream_t gs = (g == 0) ? s : w->sub_stream[g - 1];
    dyson_status st = DYSON_OK;
    if (g > 0) {
      (void)hipSetDevice(p->ctx->device);
      gw->d = w->d;
      gw->d_fkey = w->d_fkey;
      gw->pending = DYSON_OK;
      gw->stat_inner = 0;
      gw->stat_inner_max = 0;
      gw->stat_restarts = 0;
      gw->stat_capped = 0;
      gw->fac_g[0] = gw->fac_g[1] = -1000;
      gw->prof.reset();
      gw->prof.on = w->prof.on;
      launch_zero(gw->gacc, V * sizeof(double), gs);
      if (gw->prof.on) launch_zero(gw->d_prof, 8 * sizeof(unsigned long long), gs);
    }
    Run gr{p, gw, K, gs};
    for (int l : groups[g]) {
      if (st != DYSON_OK) break;
      if (abort && abort()) {
        st = fail(DYSON_ECANCELLED, "cancelled");
        break;
      }
      auto tl = std::chrono::steady_clock::now();
      st = P.opts.interface_lanczos ? gr.lanczos_level_iface(l, &lsteps_of[l])
                                    : gr.lanczos_level(l, &lsteps_of[l]);
      if (verbose) {
        int lmax = 0;
        for (int v : lsteps_of[l]) lmax = std::max(lmax, v);
        std::fprintf(stderr, "[dyson] level %d (group %d): %d domains x %d freqs, max steps %d, %.1f ms\n",
                     l, g, p->lv[l].n, K, lmax,
                     std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tl).count());
        std::fflush(stderr);
      }
      if (st == DYSON_OK && gw->pending != DYSON_OK) {
        st = gw->pending;
        g_err = st == DYSON_ENOCONV ? "inner COCG solve hit max_inner_iters"
                                    : "Lanczos breakdown persisted after restarts";
      }
    }
    if (hipStreamSynchronize(gs) != hipSuccess && st == DYSON_OK)
      st = fail(DYSON_EDEVICE, "level group stream failed");
    gst[g] = st;
    if (st != DYSON_OK) gerr[g] = g_err;
  };
  {
    std::vector<std::thread> th;
    for (int g = 1; g < G; ++g) th.emplace_back(run_group, g);
    run_group(0);
    for (auto& t : th) t.join();
  }
  for (int g = 0; g < G; ++g)
    if (gst[g] != DYSON_OK) return fail(gst[g], gerr[g]);
  // fixed order: the main group accumulated into gacc, the others follow
  if (G > 1) {
    LzArgs all = run.lz_args(0);  // level 0: one domain over every tile
    for (int g = 1; g < G; ++g) launch_add_into(all, K, w->sub[g - 1]->gacc, w->gacc, s);
    HIPC(hipGetLastError());
  }
  // sampled error estimate: G_ii against e_i^T H^{-1} e_i from a direct
  // inner solve of H x = e_i (eq. (14)) at the check sites, every frequency
  double est = 0.0;
  const int nchk = std::min<int>(P.opts.check_sites, (int)p->check_pos.size());
  if (nchk > 0) {
    const dyson_status saved = w->pending;
    w->pending = DYSON_OK;
    launch_zero(w->d_err, sizeof(double), s);
    void* fac0 = nullptr;
    CHECKED(run.factors_for(0, 0, &fac0));
    for (int c = 0; c < nchk; ++c) {
      launch_unit_vector(p->geom, K, p->check_pos[c], w->rhs, s);
      CHECKED(run.cocg(0, 0, fac0, w->rhs, w->xH, false));
      launch_sample_err(p->geom, K, p->check_pos[c], w->xH, w->gacc, w->d_err, s);
    }
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(&est, w->d_err, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (w->pending != DYSON_OK) est = std::nan("");  // the check itself did not converge
    w->pending = saved;
  }
  int max_rank_used = 0;
  long long lsteps = 0;
  for (auto& v : lsteps_of)
    for (int x : v) max_rank_used = std::max(max_rank_used, x), lsteps += x;
  for (int g = 1; g < G; ++g) {
    Work* sw = w->sub[g - 1].get();
    w->stat_inner += sw->stat_inner;
    w->stat_inner_max = std::max(w->stat_inner_max, sw->stat_inner_max);
    w->stat_restarts += sw->stat_restarts;
    w->stat_capped += sw->stat_capped;
  }
  // a8: scatter each slice to natural order
  for (int j = 0, k0 = 0; j < n; k0 += sl[j].K, ++j)
    launch_from_tile(p->geom, sl[j].K, w->gacc + (size_t)k0 * NP * 2, sl[j].G, s);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->levels = (int)P.levels.size();
    rep->max_rank_used = max_rank_used;
    rep->lanczos_steps = lsteps;
    rep->inner_iters = w->stat_inner;
    rep->inner_iters_max = w->stat_inner_max;
    rep->restarts = w->stat_restarts;
    rep->truncated = w->stat_capped > 0 ? 1 : 0;
    rep->capped_items = w->stat_capped;
    rep->batches = 1;
    rep->hbm_bytes = w->bytes;
    rep->est_rel_err = est;
    if (w->prof.on) {
      for (int g = 0; g < G; ++g) {
        Work* gw = (g == 0) ? w : w->sub[g - 1].get();
        unsigned long long wb[8];
        HIPC(hipMemcpy(wb, gw->d_prof, sizeof(wb), hipMemcpyDeviceToHost));
        double ms_c[4] = {0, 0, 0, 0};
        for (auto& m : gw->prof.marks) {
          float ms = 0;
          if (hipEventElapsedTime(&ms, m.second.first, m.second.second) == hipSuccess)
            ms_c[m.first] += ms;
        }
        for (int c = 0; c < 4; ++c) {
          // the timed sample scaled to all of the class's launches
          if (gw->prof.timed[c] > 0)
            rep->kern_ms[c] += ms_c[c] * (double)gw->prof.launches[c] / (double)gw->prof.timed[c];
          rep->kern_launches[c] += gw->prof.launches[c];
          rep->kern_bytes[c] += (double)wb[c];
        }
      }
    }
    rep->t_total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return w->pending;
}

}  // namespace dyson

// ================================================================ C ABI
extern "C" {

const char* dyson_last_error(void) { return g_err.c_str(); }
const char* dyson_version(void) { return "dyson-mi355x 0.2 (gfx950)"; }

dyson_status dyson_create(dyson_ctx** ctx, int device, size_t hbm_budget,
                          const dyson_allocator* allocator) {
  if (!ctx) return fail(DYSON_EINVAL, "null ctx");
  int n = 0;
  HIPC(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(DYSON_EINVAL, "device ordinal out of range");
  if (allocator && (!allocator->alloc || !allocator->free))
    return fail(DYSON_EINVAL, "allocator needs both alloc and free");
  HIPC(hipSetDevice(device));
  auto c = std::make_unique<dyson_ctx>();
  c->device = device;
  if (allocator) {
    c->has_alloc = true;
    c->alloc = *allocator;
  }
  if (hbm_budget == 0) {
    size_t fr = 0, tot = 0;
    HIPC(hipMemGetInfo(&fr, &tot));
    hbm_budget = fr / 10 * 9;
  }
  c->budget = hbm_budget;
  CHECKED(noalloc_init(device));
  *ctx = c.release();
  return DYSON_OK;
}

dyson_status dyson_destroy(dyson_ctx* ctx) {
  if (!ctx) return DYSON_OK;
  if (ctx->live_plans.load() > 0)
    return fail(DYSON_EBUSY, "context has plans that are not yet destroyed");
  delete ctx;  // stops the server first (serve.cpp)
  return DYSON_OK;
}

dyson_status dyson_plan_create(dyson_ctx* ctx, const dyson_lattice* lat, const dyson_opts* opts,
                               dyson_plan** out) {
  if (!lat || !out) return fail(DYSON_EINVAL, "null argument");
  dyson_opts o = merge_opts(opts);
  auto p = std::make_unique<dyson_plan>();
  std::string e = build_plan(*lat, o, p->hp);
  if (!e.empty()) return fail(DYSON_EINVAL, e);
  p->ctx = ctx;
  const HostPlan& P = p->hp;
  p->kcap = 1;
  p->nmax = 1;
  for (const auto& L : P.levels) {
    p->nmax = std::max(p->nmax, L.n_nodes);
    for (int m : L.m) p->kcap = std::max(p->kcap, step_cap(m, o) + 1);
  }
  p->hstride = p->kcap + 1;
  // tiles of each level that hold its interface sites (the interface form's
  // compact basis is sized for the largest count)
  for (size_t lev = 0; lev < P.levels.size(); ++lev) {
    int n = 0;
    for (int t = 0; t < P.T; ++t) {
      bool has = false;
      for (int q = 0; q < P.S && !has; ++q) {
        const size_t pos = (size_t)t * P.S + q;
        has = P.kind[pos] == KIND_SEP && P.depth[pos] == (int)lev;
      }
      n += has;
    }
    p->nimax = std::max(p->nimax, n);
  }
  if (ctx) {
    HIPC(hipSetDevice(ctx->device));
    const size_t TS = (size_t)P.T * P.S;
    CHECKED(dalloc(&p->d_nbr, P.nbr.size()));
    CHECKED(dalloc(&p->d_kind, TS));
    CHECKED(dalloc(&p->d_depth, TS));
    CHECKED(dalloc(&p->d_site_of, TS));
    CHECKED(dalloc(&p->d_pos_of, (size_t)P.N));
    HIPC(hipMemcpy(p->d_nbr, P.nbr.data(), P.nbr.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(p->d_kind, P.kind.data(), TS, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(p->d_depth, P.depth.data(), TS, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(p->d_site_of, P.site_of.data(), TS * sizeof(int), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(p->d_pos_of, P.pos_of.data(), (size_t)P.N * sizeof(int), hipMemcpyHostToDevice));
    for (size_t lev = 0; lev < P.levels.size(); ++lev) {
      const auto& L = P.levels[lev];
      DevLevel d;
      d.n = L.n_nodes;
      // tiles that hold interface sites of the level, grouped by domain: the
      // interface form's Lanczos vectors vanish on every other tile
      std::vector<int> itl, ilo(L.n_nodes), ihi(L.n_nodes);
      for (int nd = 0; nd < L.n_nodes; ++nd) {
        ilo[nd] = (int)itl.size();
        for (int t = L.tile_lo[nd]; t < L.tile_hi[nd]; ++t) {
          bool has = false;
          for (int q = 0; q < P.S && !has; ++q) {
            const size_t pos = (size_t)t * P.S + q;
            has = P.kind[pos] == KIND_SEP && P.depth[pos] == (int)lev;
          }
          if (has) itl.push_back(t);
        }
        ihi[nd] = (int)itl.size();
      }
      d.n_itiles = (int)itl.size();
      std::vector<int> tpos(P.T, -1);
      for (size_t q = 0; q < itl.size(); ++q) tpos[itl[q]] = (int)q;
      CHECKED(dalloc(&d.itpos, (size_t)P.T));
      HIPC(hipMemcpy(d.itpos, tpos.data(), P.T * sizeof(int), hipMemcpyHostToDevice));
      CHECKED(dalloc(&d.itiles, std::max<size_t>(itl.size(), 1)));
      CHECKED(dalloc(&d.ilo, (size_t)L.n_nodes));
      CHECKED(dalloc(&d.ihi, (size_t)L.n_nodes));
      if (!itl.empty())
        HIPC(hipMemcpy(d.itiles, itl.data(), itl.size() * sizeof(int), hipMemcpyHostToDevice));
      HIPC(hipMemcpy(d.ilo, ilo.data(), L.n_nodes * sizeof(int), hipMemcpyHostToDevice));
      HIPC(hipMemcpy(d.ihi, ihi.data(), L.n_nodes * sizeof(int), hipMemcpyHostToDevice));
      std::vector<int> cap(L.n_nodes);
      for (int i = 0; i < L.n_nodes; ++i) cap[i] = step_cap(L.m[i], o);
      CHECKED(dalloc(&d.tile_node, (size_t)P.T));
      CHECKED(dalloc(&d.tlo, (size_t)L.n_nodes));
      CHECKED(dalloc(&d.thi, (size_t)L.n_nodes));
      CHECKED(dalloc(&d.mcap, (size_t)L.n_nodes));
      CHECKED(dalloc(&d.m, (size_t)L.n_nodes));
      HIPC(hipMemcpy(d.tile_node, L.tile_node.data(), P.T * sizeof(int), hipMemcpyHostToDevice));
      HIPC(hipMemcpy(d.tlo, L.tile_lo.data(), L.n_nodes * sizeof(int), hipMemcpyHostToDevice));
      HIPC(hipMemcpy(d.thi, L.tile_hi.data(), L.n_nodes * sizeof(int), hipMemcpyHostToDevice));
      HIPC(hipMemcpy(d.mcap, cap.data(), L.n_nodes * sizeof(int), hipMemcpyHostToDevice));
      HIPC(hipMemcpy(d.m, L.m.data(), L.n_nodes * sizeof(int), hipMemcpyHostToDevice));
      p->lv.push_back(d);
    }
    ctx->live_plans.fetch_add(1);
    p->geom = TileGeom{P.T, P.S, P.sx, P.sy, P.N, P.t, p->d_nbr, p->d_kind, p->d_depth,
                       p->d_site_of, p->d_pos_of, P.s, P.dim,
                       (unsigned)(0x100000000ULL / (unsigned)P.s) + 1u};
    // check sites: a top-level interface site and a subdomain site, both
    // found from the middle of the lattice in natural order
    if (!P.levels.empty()) {
      auto find = [&](int from, auto pred) {
        for (int q = 0; q < P.N; ++q) {
          const int i = (from + q) % P.N;
          if (pred(P.pos_of[i])) return P.pos_of[i];
        }
        return -1;
      };
      const int a = find(P.N / 2, [&](int pos) { return P.kind[pos] == KIND_SEP && P.depth[pos] == 0; });
      const int b = find((P.N / 2 + P.N / 3) % P.N, [&](int pos) { return P.kind[pos] == KIND_LEAF; });
      if (a >= 0) p->check_pos.push_back(a);
      if (b >= 0) p->check_pos.push_back(b);
    }
  }
  *out = p.release();
  return DYSON_OK;
}

dyson_status dyson_plan_trim(dyson_plan* p) {
  if (!p || !p->ctx) return fail(DYSON_EINVAL, "plan has no device context");
  HIPC(hipSetDevice(p->ctx->device));
  free_work(&p->main, nullptr);
  return DYSON_OK;
}

dyson_status dyson_plan_destroy(dyson_plan* p) {
  if (!p) return DYSON_OK;
  if (p->live_requests.load() > 0)
    return fail(DYSON_EBUSY, "plan has requests that are not yet released");
  if (p->ctx) {
    (void)hipSetDevice(p->ctx->device);
    dyson::serve_forget_plan(p->ctx, p);
    free_work(&p->main, nullptr);
    for (auto& d : p->lv) {
      (void)hipFree(d.tile_node);
      (void)hipFree(d.tlo);
      (void)hipFree(d.thi);
      (void)hipFree(d.mcap);
      (void)hipFree(d.m);
      (void)hipFree(d.itiles);
      (void)hipFree(d.ilo);
      (void)hipFree(d.ihi);
      (void)hipFree(d.itpos);
    }
    (void)hipFree(p->d_nbr);
    (void)hipFree(p->d_kind);
    (void)hipFree(p->d_depth);
    (void)hipFree(p->d_site_of);
    (void)hipFree(p->d_pos_of);
    p->ctx->live_plans.fetch_sub(1);
  }
  delete p;
  return DYSON_OK;
}

dyson_status dyson_plan_get_info(const dyson_plan* p, dyson_plan_info* info) {
  if (!p || !info) return fail(DYSON_EINVAL, "null argument");
  std::memset(info, 0, sizeof(*info));
  const HostPlan& P = p->hp;
  info->n_sites = P.N;
  info->n_tiles = P.T;
  info->tile_sites = P.S;
  info->levels = (int)P.levels.size();
  for (size_t l = 0; l < P.levels.size() && l < 32; ++l) {
    info->n_nodes[l] = P.levels[l].n_nodes;
    long long sm = 0;
    int mx = 0;
    for (int m : P.levels[l].m) sm += m, mx = std::max(mx, m);
    info->max_m[l] = mx;
    info->sum_m[l] = sm;
  }
  return DYSON_OK;
}

dyson_status dyson_plan_get_maps(const dyson_plan* p, int* h_depth, int* h_is_sep, int* h_tile) {
  if (!p) return fail(DYSON_EINVAL, "null plan");
  const HostPlan& P = p->hp;
  for (int i = 0; i < P.N; ++i) {
    const int pos = P.pos_of[i];
    if (h_depth) h_depth[i] = P.depth[pos];
    if (h_is_sep) h_is_sep[i] = P.kind[pos] == KIND_SEP ? 1 : 0;
    if (h_tile) h_tile[i] = pos / P.S;
  }
  return DYSON_OK;
}

dyson_status dyson_plan_get_domains(const dyson_plan* p, int level, int* h_m, int* h_cap) {
  if (!p) return fail(DYSON_EINVAL, "null plan");
  const HostPlan& P = p->hp;
  if (level < 0 || level >= (int)P.levels.size()) return fail(DYSON_EINVAL, "bad level");
  const LevelTable& L = P.levels[level];
  for (int i = 0; i < L.n_nodes; ++i) {
    if (h_m) h_m[i] = L.m[i];
    if (h_cap) h_cap[i] = step_cap(L.m[i], P.opts);
  }
  return DYSON_OK;
}

dyson_status dyson_footprint(const dyson_plan* p, int K, size_t* bytes) {
  if (!p || !bytes || K < 1) return fail(DYSON_EINVAL, "bad argument");
  *bytes = work_bytes(p, K);
  return DYSON_OK;
}

dyson_status dyson_assemble(dyson_plan* p, int K, const double* d_V, const double* d_omega,
                            const double* d_sigma, double* d_d, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  Work* w = p ? &p->main : nullptr;
  CHECKED(begin_call(p, w, K, s));
  launch_assemble(p->geom, K, p->hp.mu, d_V, d_omega, 0, d_sigma, w->d, s);
  launch_from_tile(p->geom, K, w->d, d_d, s);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
  return DYSON_OK;
}

dyson_status dyson_leaf_diag(dyson_plan* p, int K, const double* d_d, double* d_Gleaf,
                             void* stream) {
  hipStream_t s = (hipStream_t)stream;
  Work* w = p ? &p->main : nullptr;
  CHECKED(begin_call(p, w, K, s));
  launch_to_tile(p->geom, K, d_d, w->d, 1.0, s);
  const size_t V = (size_t)K * p->hp.T * p->hp.S * 2;
  launch_zero(w->gacc, V * sizeof(double), s);
  launch_factor_diag(p->geom, K, w->d, w->fac64, w->gacc, s);
  launch_from_tile(p->geom, K, w->gacc, d_Gleaf, s);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
  return DYSON_OK;
}

dyson_status dyson_xmatvec(dyson_plan* p, int level, int K, const double* d_d, const double* d_q,
                           double* d_u, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  Work* w = p ? &p->main : nullptr;
  CHECKED(begin_call(p, w, K, s));
  if (level < 0 || level >= (int)p->hp.levels.size()) return fail(DYSON_EINVAL, "bad level");
  launch_to_tile(p->geom, K, d_d, w->d, 1.0, s);
  const size_t V = (size_t)K * p->hp.T * p->hp.S * 2;
  launch_to_tile(p->geom, K, d_q, w->R, 0.0, s);
  launch_zero(w->xH, V * sizeof(double), s);
  Run run{p, w, K, s};
  CHECKED(run.reset_items(level));
  CHECKED(run.xmatvec(level, w->R, w->xH));
  launch_from_tile(p->geom, K, w->xH, d_u, s);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
  return w->pending;
}

dyson_status dyson_correct_level(dyson_plan* p, int level, int K, const double* d_d,
                                 double* d_Gacc, int* h_steps, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  Work* w = p ? &p->main : nullptr;
  CHECKED(begin_call(p, w, K, s));
  if (level < 0 || level >= (int)p->hp.levels.size()) return fail(DYSON_EINVAL, "bad level");
  launch_to_tile(p->geom, K, d_d, w->d, 1.0, s);
  launch_to_tile(p->geom, K, d_Gacc, w->gacc, 0.0, s);
  Run run{p, w, K, s};
  std::vector<int> steps;
  CHECKED(p->hp.opts.interface_lanczos ? run.lanczos_level_iface(level, &steps)
                                        : run.lanczos_level(level, &steps));
  launch_from_tile(p->geom, K, w->gacc, d_Gacc, s);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
  if (h_steps) std::memcpy(h_steps, steps.data(), steps.size() * sizeof(int));
  return w->pending;
}

dyson_status dyson_solve(dyson_plan* p, int K, const double* d_V, const double* d_omega,
                         const double* d_sigma, double* d_G, void* stream, dyson_report* rep) {
  if (!p || !p->ctx) return fail(DYSON_EINVAL, "plan has no device context");
  if (K < 1 || K > kMaxFreqs) return fail(DYSON_EINVAL, "K must be in [1, 65535]");
  hipStream_t s = (hipStream_t)stream;
  Work* w = &p->main;
  HIPC(hipSetDevice(p->ctx->device));
  CHECKED(ensure_work(p, w, K, s));
  Slice sl{K, d_V, d_omega, d_sigma, d_G, 0};
  CHECKED(validate_slices(p, w, &sl, 1, s));
  return run_solve(p, w, &sl, 1, s, rep, nullptr);
}

dyson_status dyson_solve_host(dyson_plan* p, int K, const double* h_V, const double* h_omega,
                              const double* h_sigma, double* h_G, void* stream,
                              dyson_report* rep) {
  if (!p || !p->ctx) return fail(DYSON_EINVAL, "plan has no device context");
  if (K < 1 || K > kMaxFreqs) return fail(DYSON_EINVAL, "K must be in [1, 65535]");
  if (!h_V || !h_omega || !h_sigma || !h_G) return fail(DYSON_EINVAL, "null input or output pointer");
  hipStream_t s = (hipStream_t)stream;
  HIPC(hipSetDevice(p->ctx->device));
  const size_t N = (size_t)p->hp.N;
  const size_t bV = N * 8, bOm = (size_t)K * 8, bSig = (size_t)K * N * 16;
  // one staging block for the inputs and G, freed before returning
  char* buf = (char*)dev_alloc(p->ctx, bV + bOm + 2 * bSig + 1024, s);
  if (!buf) return fail(DYSON_ENOMEM, "device staging of the host arrays failed");
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  double* dV = (double*)buf;
  double* dOm = (double*)(buf + al(bV));
  double* dSig = (double*)(buf + al(bV) + al(bOm));
  double* dG = (double*)(buf + al(bV) + al(bOm) + al(bSig));
  const auto t0 = std::chrono::steady_clock::now();
  auto go = [&]() -> dyson_status {
    HIPC(hipMemcpyAsync(dV, h_V, bV, hipMemcpyHostToDevice, s));
    HIPC(hipMemcpyAsync(dOm, h_omega, bOm, hipMemcpyHostToDevice, s));
    HIPC(hipMemcpyAsync(dSig, h_sigma, bSig, hipMemcpyHostToDevice, s));
    Work* w = &p->main;
    CHECKED(ensure_work(p, w, K, s));
    Slice sl{K, dV, dOm, dSig, dG, 0};
    CHECKED(validate_slices(p, w, &sl, 1, s));
    CHECKED(run_solve(p, w, &sl, 1, s, rep, nullptr));
    HIPC(hipMemcpyAsync(h_G, dG, bSig, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (rep)  // host to host: the copies are part of the call's time
      rep->t_total_ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return DYSON_OK;
  };
  const dyson_status st = go();
  (void)hipStreamSynchronize(s);
  const std::string msg = g_err;
  dev_free(p->ctx, buf, s);
  g_err = msg;
  return st;
}

dyson_status dyson_autotune(dyson_ctx* ctx, const dyson_lattice* lat, const dyson_opts* base,
                            int K, const double* d_V, const double* d_omega,
                            const double* d_sigma, dyson_opts* best, double* rate) {
  if (!ctx || !lat || !best || K < 1 || K > kMaxFreqs) return fail(DYSON_EINVAL, "bad argument");
  if (!d_V || !d_omega || !d_sigma) return fail(DYSON_EINVAL, "null input pointer");
  const dyson_opts b0 = merge_opts(base);
  std::vector<int> edges = (lat->dim == 3) ? std::vector<int>DYSON_AUTOTUNE_EDGES_3D
                                            : std::vector<int>DYSON_AUTOTUNE_EDGES_2D;
  const std::vector<int> streams = DYSON_AUTOTUNE_LEVEL_STREAMS;
  std::vector<int> forms = DYSON_AUTOTUNE_FORMS;
  if (b0.max_rank > 0) forms = {0};  // a truncated rank exists in the X form only
  long long n = 1;
  for (int a = 0; a < 3; ++a) n *= std::max(1, lat->L[a]);
  HIPC(hipSetDevice(ctx->device));
  double* G = (double*)dev_alloc(ctx, (size_t)K * n * 16, nullptr);
  if (!G) return fail(DYSON_ENOMEM, "probe output allocation failed");
  double best_s = -1.0;
  dyson_status last = DYSON_EINVAL;
  std::string last_err = "no valid candidate";
  for (int e : edges)
    for (int ls : streams)
    for (int f : forms) {
      dyson_opts o = b0;
      o.leaf_edge = e;
      o.level_streams = ls;
      o.interface_lanczos = f;
      o.profile = 0;
      dyson_plan* p = nullptr;
      if (dyson_plan_create(ctx, lat, &o, &p) != DYSON_OK) continue;  // e.g. periodic extent
      Work* w = &p->main;
      dyson_status st = ensure_work(p, w, K, nullptr);
      Slice sl{K, d_V, d_omega, d_sigma, G, 0};
      if (st == DYSON_OK) st = validate_slices(p, w, &sl, 1, nullptr);
      if (st == DYSON_OK) {
        (void)hipDeviceSynchronize();
        auto t0 = std::chrono::steady_clock::now();
        st = run_solve(p, w, &sl, 1, nullptr, nullptr, nullptr);
        const double secs =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (st == DYSON_OK && (best_s < 0 || secs < best_s)) {
          best_s = secs;
          *best = o;
        }
      }
      if (st != DYSON_OK) {
        last = st;
        last_err = g_err;
      }
      dyson_plan_destroy(p);
      if (st == DYSON_EINVAL) break;  // the probe inputs themselves are invalid
    }
  dev_free(ctx, G, nullptr);
  if (best_s < 0) return fail(last, last_err);
  if (rate) *rate = (double)n * K / best_s;
  return DYSON_OK;
}

dyson_status dyson_solve_z(dyson_plan* p, int K, const double* d_V, const double* d_z,
                           const double* d_sigma, double* d_G, void* stream, dyson_report* rep) {
  if (!p || !p->ctx) return fail(DYSON_EINVAL, "plan has no device context");
  if (K < 1 || K > kMaxFreqs) return fail(DYSON_EINVAL, "K must be in [1, 65535]");
  hipStream_t s = (hipStream_t)stream;
  Work* w = &p->main;
  HIPC(hipSetDevice(p->ctx->device));
  CHECKED(ensure_work(p, w, K, s));
  Slice sl{K, d_V, d_z, d_sigma, d_G, 1};
  CHECKED(validate_slices(p, w, &sl, 1, s));
  return run_solve(p, w, &sl, 1, s, rep, nullptr);
}

}  // extern "C"
