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
#include <vector>

#include "../../include/dyson.h"
#include "kernels.h"
#include "plan.h"

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

struct DevLevel {
  int n = 0;
  int* tile_node = nullptr;
  int* tlo = nullptr;
  int* thi = nullptr;
  int* mcap = nullptr;
};

// Event-timed kernel classes (report.kern_*).
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
  size_t used = 0;
  long long launches[4] = {0, 0, 0, 0};
  double bytes[4] = {0, 0, 0, 0};
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void reset() {
    used = 0;
    marks.clear();
    for (int c = 0; c < 4; ++c) launches[c] = 0, bytes[c] = 0;
  }
  ~Prof() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct dyson_ctx {
  int device = 0;
};

struct dyson_plan {
  dyson_ctx* ctx = nullptr;
  HostPlan hp;
  TileGeom geom{};
  int* d_nbr = nullptr;
  uint8_t* d_kind = nullptr;
  uint8_t* d_depth = nullptr;
  int* d_site_of = nullptr;
  int* d_pos_of = nullptr;
  std::vector<DevLevel> lv;
  int kcap = 1;     // largest Lanczos step cap + 1 (basis vectors)
  int nmax = 1;     // most domains on one level
  // workspace for up to Kcap frequencies
  int Kcap = 0;
  std::vector<void*> allocs;
  double *d = nullptr, *gacc = nullptr, *xB = nullptr, *xH = nullptr, *r = nullptr, *z = nullptr,
         *p0 = nullptr, *p1 = nullptr, *s = nullptr, *rhs = nullptr, *R = nullptr, *Q = nullptr;
  void* fac[2] = {nullptr, nullptr};
  double* fac64 = nullptr;  // complex128 leaf factors written with the leaf diagonal
  int fac_g[2] = {-1000, -1000};
  double* partial = nullptr;
  double *hpart = nullptr, *h = nullptr;
  int hstride = 1;
  CocgState cst{};
  int *lz_stopped = nullptr, *lz_steps = nullptr;
  double* Dl = nullptr;     // diagonal correction of the level being run
  double *lz_alpha = nullptr, *lz_beta = nullptr, *lz_unorm2 = nullptr, *lz_umax2 = nullptr,
         *lz_scal = nullptr;
  int* d_count = nullptr;
  double* rho2 = nullptr;   // inner solves: r^T z of the last two iterations per item
  double* partS = nullptr;  // inner solves: per-unit p^T A p
  std::vector<int> pred;    // predicted inner iterations per (level, graph) for polling
  int* h_count = nullptr;  // pinned
  unsigned long long* d_prof = nullptr;
  unsigned long long* d_wprof = nullptr;  // [4][K*nmax] per-item byte counts (profiling):
                                          // inner solves in [0,2), Lanczos in [2,4)
  uint64_t* d_fkey = nullptr;
  Prof prof;
  // run statistics of the current call
  long long stat_inner = 0;
  int stat_inner_max = 0;
  int stat_restarts = 0;
  int stat_capped = 0;      // items stopped by the step cap before exhaustion
  dyson_status pending = DYSON_OK;
};

namespace {

// Lanczos step cap of a domain with interface size m: the paper allows 5-10
// steps beyond m for m ~ 100; bilinear Lanczos in floating point needs more
// as m grows (m + 11 observed at m = 128), so the allowance scales as m/8.
int step_cap(int m, const dyson_opts& o) {
  int c = m + std::max(o.extra_steps, (m + 7) / 8);
  if (o.max_rank > 0) c = std::min(c, o.max_rank);
  return c;
}

void free_workspace(dyson_plan* p) {
  for (void* a : p->allocs) (void)hipFree(a);
  p->allocs.clear();
  if (p->h_count) (void)hipHostFree(p->h_count);
  p->h_count = nullptr;
  p->Kcap = 0;
  p->fac_g[0] = p->fac_g[1] = -1000;
}

template <typename T>
dyson_status walloc(dyson_plan* p, T** ptr, size_t n) {
  CHECKED(dalloc(ptr, n));
  p->allocs.push_back((void*)*ptr);
  return DYSON_OK;
}

dyson_status ensure_workspace(dyson_plan* p, int K) {
  if (K <= p->Kcap) return DYSON_OK;
  HIPC(hipSetDevice(p->ctx->device));
  free_workspace(p);
  const HostPlan& P = p->hp;
  const size_t NP = (size_t)P.T * P.S;
  const size_t V = (size_t)K * NP * 2;  // doubles per complex vector
  CHECKED(walloc(p, &p->d, V));
  CHECKED(walloc(p, &p->gacc, V));
  CHECKED(walloc(p, &p->xB, V));
  CHECKED(walloc(p, &p->xH, V));
  CHECKED(walloc(p, &p->r, V));
  CHECKED(walloc(p, &p->z, V));
  CHECKED(walloc(p, &p->p0, V));
  CHECKED(walloc(p, &p->p1, V));
  CHECKED(walloc(p, &p->s, V));
  CHECKED(walloc(p, &p->rhs, V));
  CHECKED(walloc(p, &p->R, V));
  CHECKED(walloc(p, &p->Dl, V));
  const int nq = P.levels.empty() ? 1 : (p->kcap + 1);
  CHECKED(walloc(p, &p->Q, V * (size_t)nq));
  const size_t fe = (size_t)K * P.T * P.sy * P.sx * P.sx * 2;  // reals per factor set
  for (int i = 0; i < 2; ++i) {
    if (P.opts.precision == DYSON_PREC_FP64) {
      double* f;
      CHECKED(walloc(p, &f, fe));
      p->fac[i] = f;
      if (i == 0) p->fac64 = f;  // the leaf factors are the deepest B preconditioner
      continue;
    }
    if (P.opts.precision == DYSON_PREC_MIXED) {
      float* f;
      CHECKED(walloc(p, &f, fe));
      p->fac[i] = f;
    } else if (P.opts.precision == DYSON_PREC_MIXED16) {
      uint16_t* f;
      CHECKED(walloc(p, &f, fe));
      p->fac[i] = f;
    } else {
      double* f;
      CHECKED(walloc(p, &f, fe));
      p->fac[i] = f;
    }
  }
  if (P.opts.precision != DYSON_PREC_FP64) CHECKED(walloc(p, &p->fac64, fe));
  CHECKED(walloc(p, &p->partial, (size_t)K * P.T * 4));
  CHECKED(walloc(p, &p->hpart, (size_t)K * P.T * p->hstride * 2));
  const size_t ni = (size_t)K * p->nmax;
  CHECKED(walloc(p, &p->h, ni * p->hstride * 2));
  CHECKED(walloc(p, &p->cst.done, ni));
  CHECKED(walloc(p, &p->cst.iters, ni));
  CHECKED(walloc(p, &p->cst.bn2, ni));
  CHECKED(walloc(p, &p->rho2, ni * 4));
  CHECKED(walloc(p, &p->partS, (size_t)K * P.T * 2));
  CHECKED(walloc(p, &p->lz_stopped, ni));
  CHECKED(walloc(p, &p->lz_steps, ni));
  CHECKED(walloc(p, &p->lz_alpha, ni * 2));
  CHECKED(walloc(p, &p->lz_beta, ni * 2));
  CHECKED(walloc(p, &p->lz_unorm2, ni));
  CHECKED(walloc(p, &p->lz_umax2, ni));
  CHECKED(walloc(p, &p->lz_scal, ni * 2));
  CHECKED(walloc(p, &p->d_count, 4));
  CHECKED(walloc(p, &p->d_prof, 8));
  CHECKED(walloc(p, &p->d_wprof, 4 * ni));
  HIPC(hipMemset(p->d_wprof, 0, 4 * ni * sizeof(unsigned long long)));
  CHECKED(walloc(p, &p->d_fkey, (size_t)K));
  HIPC(hipHostMalloc((void**)&p->h_count, 4 * sizeof(int), hipHostMallocDefault));
  p->Kcap = K;
  return DYSON_OK;
}

}  // namespace

namespace {

// ----------------------------------------------------------- the solver
struct Run {
  dyson_plan* p;
  int K;
  hipStream_t s;
  const HostPlan& P() const { return p->hp; }

  // Time a launch when profiling: class c, algorithmic bytes b.
  template <typename Fn>
  void timed(int c, Fn fn) {
    Prof& pr = p->prof;
    // profile = 1: events around the inner-solve update kernel only (the
    // dominant kernel); profile >= 2: around every timed kernel class
    if (!pr.on || (P().opts.profile < 2 && c != 0)) {
      if (pr.on) pr.launches[c] += 1;
      fn();
      return;
    }
    hipEvent_t a = pr.get(), b = pr.get();
    (void)hipEventRecord(a, s);
    fn();
    (void)hipEventRecord(b, s);
    pr.marks.push_back({c, {a, b}});
    pr.launches[c] += 1;
  }

  dyson_status count_open(const int* flags, int n, int* out) {
    launch_count_open(flags, n, p->d_count, s);
    HIPC(hipMemcpyAsync(p->h_count, p->d_count, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    *out = p->h_count[0];
    return DYSON_OK;
  }

  // Factor the tile blocks of graph g (cached in one of two slots).
  dyson_status factors_for(int g, int level, void** fac) {
    for (int i = 0; i < 2; ++i)
      if (p->fac_g[i] == g) {
        *fac = p->fac[i];
        return DYSON_OK;
      }
    // evict the slot not holding the other graph of this level
    int slot = (p->fac_g[0] == g + 1 || p->fac_g[0] == g - 1) ? 1 : 0;
    (void)level;  // every tile is factored: a graph is shared by two levels
    launch_factor(p->geom, K, g, nullptr, p->d, p->fac[slot],
                  P().opts.precision == DYSON_PREC_MIXED, P().opts.precision == DYSON_PREC_MIXED16,
                  s);
    HIPC(hipGetLastError());
    p->fac_g[slot] = g;
    *fac = p->fac[slot];
    return DYSON_OK;
  }

  // COCG on graph g for every item of `level`, x = A_g^{-1} b.  Two launches
  // per iteration; the host polls the device's open-item count only near the
  // iteration count the previous solve of the same kind needed.
  dyson_status cocg(int level, int g, const void* fac, const double* b, double* x) {
    const DevLevel& L = p->lv[level];
    const HostPlan& HP = P();
    CocgLaunch c{};
    c.G = p->geom;
    c.K = K;
    c.g = g;
    c.tile_node = L.tile_node;
    c.n_nodes = L.n;
    c.item_skip = p->lz_stopped;
    c.st = p->cst;
    c.d = p->d;
    c.x = x;
    c.r = p->r;
    c.z = p->z;
    c.p_old = p->p0;
    c.p_new = p->p1;
    c.s = p->s;
    c.fac = fac;
    c.fp32 = HP.opts.precision == DYSON_PREC_MIXED;
    c.fp16 = HP.opts.precision == DYSON_PREC_MIXED16;
    c.wctr = p->prof.on ? p->d_wprof : nullptr;
    c.tlo = L.tlo;
    c.thi = L.thi;
    c.n_items = K * L.n;
    c.partS = p->partS;
    c.partU = p->partial;
    c.rho2 = p->rho2;
    c.tol2 = HP.opts.inner_tol * HP.opts.inner_tol;
    const int slot = 2 * level + (g == level ? 0 : 1);
    if ((int)p->pred.size() <= slot) p->pred.resize(slot + 1, 0);
    launch_cocg_init(c, b, s);
    launch_cocg_check(c, 0, p->d_count, s);
    const int maxit = HP.opts.max_inner_iters;
    int it = 0, open = 1;
    int check_at = std::max(1, p->pred[slot] - 1);
    while (it < maxit) {
      timed(1, [&] { launch_cocg_stencil(c, it, s); });
      timed(0, [&] { launch_cocg_update(c, it, s); });
      std::swap(c.p_old, c.p_new);
      ++it;
      if (it >= check_at || it == maxit) {
        launch_cocg_check(c, it, p->d_count, s);
        HIPC(hipMemcpyAsync(p->h_count, p->d_count, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        open = p->h_count[0];
        if (open == 0) break;
        check_at = it + (it < 8 ? 1 : 2);
      }
    }
    HIPC(hipGetLastError());
    if (open != 0) {
      p->pending = DYSON_ENOCONV;
      g_err = "inner COCG solve hit max_inner_iters";
    }
    if (p->prof.on) launch_prof_collect(p->d_wprof, K * L.n, 2, 0, p->d_prof, s);
    p->pred[slot] = it;
    p->stat_inner += it;
    p->stat_inner_max = std::max(p->stat_inner_max, it);
    return DYSON_OK;
  }

  LzArgs lz_args(int level) {
    LzArgs a{};
    a.G = p->geom;
    a.level = level;
    a.tile_node = p->lv[level].tile_node;
    a.n_nodes = p->lv[level].n;
    a.seed = P().opts.seed;
    a.fkey = p->d_fkey;
    a.stopped = p->lz_stopped;
    a.steps = p->lz_steps;
    a.alpha = p->lz_alpha;
    a.beta = p->lz_beta;
    a.unorm2 = p->lz_unorm2;
    a.umax2 = p->lz_umax2;
    a.scal = p->lz_scal;
    a.partial = p->partial;
    a.hpart = p->hpart;
    a.h = p->h;
    a.hstride = p->hstride;
    a.tlo = p->lv[level].tlo;
    a.thi = p->lv[level].thi;
    a.n_items = K * p->lv[level].n;
    a.wctr = p->prof.on ? p->d_wprof + 2 * (size_t)K * p->nmax : nullptr;
    return a;
  }

  dyson_status reset_items(int level) {
    const size_t ni = (size_t)K * p->lv[level].n;
    HIPC(hipMemsetAsync(p->lz_stopped, 0, ni * sizeof(int), s));
    HIPC(hipMemsetAsync(p->lz_steps, 0, ni * sizeof(int), s));
    HIPC(hipMemsetAsync(p->lz_beta, 0, ni * 2 * sizeof(double), s));
    return DYSON_OK;
  }

  // u = X_level q for every item (eqs. (10)-(12), solve of (10) started at w).
  dyson_status xmatvec(int level, const double* q, double* u) {
    void *facB = nullptr, *facH = nullptr;
    CHECKED(factors_for(level + 1, level, &facB));
    CHECKED(cocg(level, level + 1, facB, q, p->xB));        // w = B^{-1} q_B   (11)
    LzArgs a = lz_args(level);
    launch_lz_defect(a, K, q, p->xB, p->rhs, s);             // q - H w
    CHECKED(factors_for(level, level, &facH));
    CHECKED(cocg(level, level, facH, p->rhs, u));            // u = v - w        (10),(12)
    return DYSON_OK;
  }

  void cgs2(const LzArgs& a, const DevLevel& L, int nvec) {
    const size_t qstride = (size_t)K * P().T * P().S * 2;
    for (int pass = 0; pass < 2; ++pass) {
      timed(3, [&] { launch_cgs_dot(a, K, p->Q, qstride, nvec, p->R, s); });
      launch_cgs_reduce(a, K, L.tlo, L.thi, nvec, s);
      timed(2, [&] { launch_cgs_update(a, K, p->Q, qstride, nvec, p->R, p->Dl, s); });
    }
  }

  // One correction level: bilinear Lanczos on X for every (domain, frequency),
  // diag(Q H Q^T) gathered in Dl and added to the running diagonal at the end.
  // An item whose bilinear form breaks down is redone from a fresh start
  // vector (its partial diagonal is discarded), at most twice.
  dyson_status lanczos_level(int level, std::vector<int>* steps_out) {
    const DevLevel& L = p->lv[level];
    const HostPlan& HP = P();
    const size_t V = (size_t)K * HP.T * HP.S * 2;
    auto Qj = [&](int j) { return p->Q + (size_t)j * V; };
    CHECKED(reset_items(level));
    HIPC(hipMemsetAsync(p->Dl, 0, V * sizeof(double), s));
    LzArgs a = lz_args(level);
    const int n_items = K * L.n;
    const double brk = 1e-6;  // |r^T r| <= brk |r|^2 would give |q| >= 1e3: redo the item
    int kmax = 0;
    for (int m : HP.levels[level].m) kmax = std::max(kmax, step_cap(m, HP.opts));
    kmax = std::min(kmax, p->kcap);
    std::vector<int> st(n_items), stop(n_items);
    for (int attempt = 0; attempt < 3; ++attempt) {
      // start vector, normalized in the bilinear "norm"
      launch_lz_random(a, K, Qj(0), (uint64_t)attempt, s);
      launch_lz_scalars(a, K, L.tlo, L.thi, L.mcap, 0, 0, HP.opts.lanczos_tol, brk, s);
      launch_lz_scale(a, K, Qj(0), s);
      HIPC(hipGetLastError());
      for (int j = 0; j < kmax; ++j) {
        int open = 0;
        CHECKED(count_open(p->lz_stopped, n_items, &open));
        if (open == 0) break;
        const double* q = Qj(j);
        CHECKED(xmatvec(level, q, p->xH));
        launch_lz_alpha(a, K, q, p->xH, s);
        launch_lz_scalars(a, K, L.tlo, L.thi, L.mcap, 1, j, HP.opts.lanczos_tol, brk, s);
        launch_lz_recur(a, K, q, j > 0 ? Qj(j - 1) : nullptr, p->xH, p->R, p->Dl, s);
        cgs2(a, L, j + 1);
        launch_lz_norms(a, K, p->R, s);
        launch_lz_scalars(a, K, L.tlo, L.thi, L.mcap, 2, j, HP.opts.lanczos_tol, brk, s);
        if (j + 1 < p->kcap) launch_lz_next(a, K, p->R, Qj(j + 1), s);
        HIPC(hipGetLastError());
      }
      HIPC(hipMemcpyAsync(stop.data(), p->lz_stopped, n_items * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPC(hipMemcpyAsync(st.data(), p->lz_steps, n_items * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      int bad = 0;
      for (int i = 0; i < n_items; ++i) {
        bad += (stop[i] == 3);
        if (stop[i] == 2) p->stat_capped += 1;
      }
      if (std::getenv("DYSON_VERBOSE")) {
        int hist[5] = {0, 0, 0, 0, 0};
        for (int i = 0; i < n_items; ++i) hist[std::min(std::max(stop[i], 0), 4)]++;
        std::fprintf(stderr, "[dyson] level %d attempt %d: stop codes open=%d exhausted=%d cap=%d breakdown=%d\n",
                     level, attempt, hist[0], hist[1], hist[2], hist[3]);
      }
      if (bad == 0) break;
      if (attempt == 2) {
        p->pending = DYSON_EBREAKDOWN;
        g_err = "Lanczos breakdown persisted after restarts";
        break;
      }
      p->stat_restarts += bad;
      launch_lz_reopen(a, K, p->Dl, s);
      HIPC(hipGetLastError());
    }
    if (p->prof.on) launch_prof_collect(a.wctr, n_items, 2, 2, p->d_prof, s);
    launch_add_into(a, K, p->Dl, p->gacc, s);
    HIPC(hipGetLastError());
    if (steps_out) *steps_out = st;
    return DYSON_OK;
  }
};

dyson_status validate_inputs_host(const dyson_plan* p, int K) {
  if (!p) return fail(DYSON_EINVAL, "null plan");
  if (K < 1) return fail(DYSON_EINVAL, "K must be >= 1");
  return DYSON_OK;
}

}  // namespace

// ================================================================ C ABI
extern "C" {

const char* dyson_last_error(void) { return g_err.c_str(); }
const char* dyson_version(void) { return "dyson-mi355x 0.1 (gfx950)"; }

dyson_status dyson_create(dyson_ctx** ctx, int device) {
  if (!ctx) return fail(DYSON_EINVAL, "null ctx");
  int n = 0;
  HIPC(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(DYSON_EINVAL, "device ordinal out of range");
  HIPC(hipSetDevice(device));
  *ctx = new dyson_ctx{device};
  return DYSON_OK;
}

dyson_status dyson_destroy(dyson_ctx* ctx) {
  delete ctx;
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
    for (const auto& L : P.levels) {
      DevLevel d;
      d.n = L.n_nodes;
      std::vector<int> cap(L.n_nodes);
      for (int i = 0; i < L.n_nodes; ++i) cap[i] = step_cap(L.m[i], o);
      CHECKED(dalloc(&d.tile_node, (size_t)P.T));
      CHECKED(dalloc(&d.tlo, (size_t)L.n_nodes));
      CHECKED(dalloc(&d.thi, (size_t)L.n_nodes));
      CHECKED(dalloc(&d.mcap, (size_t)L.n_nodes));
      HIPC(hipMemcpy(d.tile_node, L.tile_node.data(), P.T * sizeof(int), hipMemcpyHostToDevice));
      HIPC(hipMemcpy(d.tlo, L.tile_lo.data(), L.n_nodes * sizeof(int), hipMemcpyHostToDevice));
      HIPC(hipMemcpy(d.thi, L.tile_hi.data(), L.n_nodes * sizeof(int), hipMemcpyHostToDevice));
      HIPC(hipMemcpy(d.mcap, cap.data(), L.n_nodes * sizeof(int), hipMemcpyHostToDevice));
      p->lv.push_back(d);
    }
    p->geom = TileGeom{P.T, P.S, P.sx, P.sy, P.N, P.t, p->d_nbr, p->d_kind, p->d_depth,
                       p->d_site_of, p->d_pos_of, P.s, P.dim};
  }
  *out = p.release();
  return DYSON_OK;
}

dyson_status dyson_plan_destroy(dyson_plan* p) {
  if (!p) return DYSON_OK;
  if (p->ctx) {
    (void)hipSetDevice(p->ctx->device);
    free_workspace(p);
    for (auto& d : p->lv) {
      (void)hipFree(d.tile_node);
      (void)hipFree(d.tlo);
      (void)hipFree(d.thi);
      (void)hipFree(d.mcap);
    }
    (void)hipFree(p->d_nbr);
    (void)hipFree(p->d_kind);
    (void)hipFree(p->d_depth);
    (void)hipFree(p->d_site_of);
    (void)hipFree(p->d_pos_of);
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

dyson_status dyson_footprint(const dyson_plan* p, int K, size_t* bytes) {
  if (!p || !bytes || K < 1) return fail(DYSON_EINVAL, "bad argument");
  const HostPlan& P = p->hp;
  const size_t NP = (size_t)P.T * P.S;
  const size_t V = (size_t)K * NP * 16;
  const size_t fsz = (P.opts.precision == DYSON_PREC_MIXED)   ? 8
                     : (P.opts.precision == DYSON_PREC_MIXED16) ? 4
                                                                : 16;
  const size_t nq = P.levels.empty() ? 1 : (size_t)(p->kcap + 1);
  size_t b = V * (12 + nq);
  b += 2 * (size_t)K * P.T * P.sy * P.sx * P.sx * fsz;
  if (P.opts.precision != DYSON_PREC_FP64) b += (size_t)K * P.T * P.sy * P.sx * P.sx * 16;
  b += (size_t)K * P.T * 2 * 16 + (size_t)K * P.T * p->hstride * 16;
  b += (size_t)K * p->nmax * p->hstride * 16 + (size_t)K * p->nmax * 200;
  *bytes = b;
  return DYSON_OK;
}

static dyson_status begin(dyson_plan* p, int K, hipStream_t s) {
  if (!p || !p->ctx) return fail(DYSON_EINVAL, "plan has no device context");
  if (K < 1) return fail(DYSON_EINVAL, "K must be >= 1");
  HIPC(hipSetDevice(p->ctx->device));
  CHECKED(ensure_workspace(p, K));
  p->pending = DYSON_OK;
  p->stat_inner = 0;
  p->stat_inner_max = 0;
  p->stat_restarts = 0;
  p->stat_capped = 0;
  p->fac_g[0] = p->fac_g[1] = -1000;  // factors depend on d, which changes per call
  launch_freq_keys(nullptr, K, p->d_fkey, s);
  return DYSON_OK;
}

// Checks eq. (1)'s inputs on the device side copy: w_k > 0, finite values,
// Im(i w_k - Sigma) > 0.  Copies to the host (validation is not in the hot loop).
static dyson_status validate_device_inputs(dyson_plan* p, int K, const double* d_V,
                                           const double* d_omega, const double* d_sigma,
                                           hipStream_t s) {
  const int N = p->hp.N;
  std::vector<double> V(N), om(K), sg((size_t)2 * K * N);
  HIPC(hipMemcpyAsync(V.data(), d_V, N * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPC(hipMemcpyAsync(om.data(), d_omega, K * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPC(hipMemcpyAsync(sg.data(), d_sigma, sg.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  for (int i = 0; i < N; ++i)
    if (!std::isfinite(V[i])) return fail(DYSON_EINVAL, "V contains a non-finite value");
  for (int k = 0; k < K; ++k) {
    if (!std::isfinite(om[k]) || om[k] <= 0) return fail(DYSON_EINVAL, "omega_k must be > 0");
    for (int i = 0; i < N; ++i) {
      const double re = sg[2 * ((size_t)k * N + i)], im = sg[2 * ((size_t)k * N + i) + 1];
      if (!std::isfinite(re) || !std::isfinite(im))
        return fail(DYSON_EINVAL, "Sigma contains a non-finite value");
      if (!(om[k] - im > 0))
        return fail(DYSON_EINVAL, "Im(i w_k - Sigma_i) must be > 0 (causal self-energy)");
    }
  }
  return DYSON_OK;
}

dyson_status dyson_assemble(dyson_plan* p, int K, const double* d_V, const double* d_omega,
                            const double* d_sigma, double* d_d, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  CHECKED(begin(p, K, s));
  launch_assemble(p->geom, K, p->hp.mu, d_V, d_omega, d_sigma, p->d, s);
  launch_from_tile(p->geom, K, p->d, d_d, s);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
  return DYSON_OK;
}

dyson_status dyson_leaf_diag(dyson_plan* p, int K, const double* d_d, double* d_Gleaf,
                             void* stream) {
  hipStream_t s = (hipStream_t)stream;
  CHECKED(begin(p, K, s));
  launch_to_tile(p->geom, K, d_d, p->d, 1.0, s);
  const size_t V = (size_t)K * p->hp.T * p->hp.S * 2;
  HIPC(hipMemsetAsync(p->gacc, 0, V * sizeof(double), s));
  launch_factor_diag(p->geom, K, p->d, p->fac64, p->gacc, s);
  launch_from_tile(p->geom, K, p->gacc, d_Gleaf, s);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
  return DYSON_OK;
}

dyson_status dyson_xmatvec(dyson_plan* p, int level, int K, const double* d_d, const double* d_q,
                           double* d_u, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  CHECKED(begin(p, K, s));
  if (level < 0 || level >= (int)p->hp.levels.size()) return fail(DYSON_EINVAL, "bad level");
  launch_to_tile(p->geom, K, d_d, p->d, 1.0, s);
  const size_t V = (size_t)K * p->hp.T * p->hp.S * 2;
  launch_to_tile(p->geom, K, d_q, p->R, 0.0, s);
  HIPC(hipMemsetAsync(p->xH, 0, V * sizeof(double), s));
  Run run{p, K, s};
  CHECKED(run.reset_items(level));
  CHECKED(run.xmatvec(level, p->R, p->xH));
  launch_from_tile(p->geom, K, p->xH, d_u, s);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
  return p->pending;
}

dyson_status dyson_correct_level(dyson_plan* p, int level, int K, const double* d_d,
                                 double* d_Gacc, int* h_steps, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  CHECKED(begin(p, K, s));
  if (level < 0 || level >= (int)p->hp.levels.size()) return fail(DYSON_EINVAL, "bad level");
  launch_to_tile(p->geom, K, d_d, p->d, 1.0, s);
  launch_to_tile(p->geom, K, d_Gacc, p->gacc, 0.0, s);
  Run run{p, K, s};
  std::vector<int> steps;
  CHECKED(run.lanczos_level(level, &steps));
  launch_from_tile(p->geom, K, p->gacc, d_Gacc, s);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
  if (h_steps) std::memcpy(h_steps, steps.data(), steps.size() * sizeof(int));
  return p->pending;
}

dyson_status dyson_solve(dyson_plan* p, int K, const double* d_V, const double* d_omega,
                         const double* d_sigma, double* d_G, void* stream, dyson_report* rep) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)stream;
  CHECKED(begin(p, K, s));
  CHECKED(validate_device_inputs(p, K, d_V, d_omega, d_sigma, s));
  const HostPlan& P = p->hp;
  p->prof.reset();
  p->prof.on = P.opts.profile != 0;
  if (p->prof.on) HIPC(hipMemsetAsync(p->d_prof, 0, 8 * sizeof(unsigned long long), s));
  Run run{p, K, s};
  launch_freq_keys(d_omega, K, p->d_fkey, s);
  // a1: diagonal of H
  launch_assemble(p->geom, K, P.mu, d_V, d_omega, d_sigma, p->d, s);
  // a3/a4: leaf factorization and diag(B^{-1})
  const size_t V = (size_t)K * P.T * P.S * 2;
  HIPC(hipMemsetAsync(p->gacc, 0, V * sizeof(double), s));
  // FP64 plans keep the leaf factors (FP64 buffers); mixed plans only take the
  // diagonal here and factor the preconditioner again in complex64
  const bool keep = P.opts.precision == DYSON_PREC_FP64;
  launch_factor_diag(p->geom, K, p->d, p->fac64, p->gacc, s);
  HIPC(hipGetLastError());
  if (keep && !P.levels.empty()) {
    // the leaf factors double as the preconditioner of the deepest B graph
    p->fac_g[0] = (int)P.levels.size();
  }
  // a5-a9: corrections bottom-up
  int max_rank_used = 0;
  long long lsteps = 0;
  const bool verbose = std::getenv("DYSON_VERBOSE") != nullptr;
  for (int l = (int)P.levels.size() - 1; l >= 0; --l) {
    std::vector<int> steps;
    auto tl = std::chrono::steady_clock::now();
    CHECKED(run.lanczos_level(l, &steps));
    int lmax = 0;
    for (int v : steps) max_rank_used = std::max(max_rank_used, v), lsteps += v, lmax = std::max(lmax, v);
    if (verbose) {
      std::fprintf(stderr, "[dyson] level %d: %d domains x %d freqs, max steps %d, %.1f ms, inner iters so far %lld\n",
                   l, p->lv[l].n, K, lmax,
                   std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tl).count(),
                   p->stat_inner);
      std::fflush(stderr);
    }
    if (p->pending != DYSON_OK) break;
  }
  // a8: scatter to natural order
  launch_from_tile(p->geom, K, p->gacc, d_G, s);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->levels = (int)P.levels.size();
    rep->max_rank_used = max_rank_used;
    rep->lanczos_steps = lsteps;
    rep->inner_iters = p->stat_inner;
    rep->inner_iters_max = p->stat_inner_max;
    rep->restarts = p->stat_restarts;
    rep->truncated = p->stat_capped > 0 ? 1 : 0;
    if (p->prof.on) {
      unsigned long long wb[8];
      HIPC(hipMemcpy(wb, p->d_prof, sizeof(wb), hipMemcpyDeviceToHost));
      for (int c = 0; c < 4; ++c) p->prof.bytes[c] = (double)wb[c];
      for (auto& m : p->prof.marks) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, m.second.first, m.second.second) == hipSuccess)
          rep->kern_ms[m.first] += ms;
      }
      for (int c = 0; c < 4; ++c) {
        rep->kern_launches[c] = p->prof.launches[c];
        rep->kern_bytes[c] = p->prof.bytes[c];
      }
    }
    rep->t_total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return p->pending;
}

}  // extern "C"
