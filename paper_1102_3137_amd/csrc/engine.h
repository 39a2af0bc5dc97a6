// Internal state shared by the blocking solver (solver.cpp) and the request
// server (serve.cpp): the device copy of a plan and the workspace one batch of
// frequencies runs in.  A plan is read-only once built; every call that
// computes runs in a Work, so several batches of one plan can be in flight on
// separate streams at once.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/dyson.h"
#include "kernels.h"
#include "plan.h"

namespace dyson {

void set_error(const std::string& msg);
extern const double kMinImMixed16;  // smallest Im H_ii of a DYSON_PREC_MIXED16 solve
const std::string& get_error();

struct DevLevel {
  int n = 0;
  int* tile_node = nullptr;
  int* tlo = nullptr;
  int* thi = nullptr;
  int* mcap = nullptr;
  int* m = nullptr;     // interface size of each domain
  int* itiles = nullptr;  // tiles holding interface sites of the level, by domain
  int* ilo = nullptr;     // [n] range of each domain in itiles
  int* ihi = nullptr;
  int* itpos = nullptr;   // [T] position of a tile in itiles, -1 if not listed
  int n_itiles = 0;
};

// Event-timed kernel classes (report.kern_*).
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
  size_t used = 0;
  long long launches[4] = {0, 0, 0, 0};
  long long timed[4] = {0, 0, 0, 0};  // launches with events around them
  double bytes[4] = {0, 0, 0, 0};
  hipEvent_t get();
  void reset();
  ~Prof();
};

struct Server;
struct SchurData;  // explicit-Schur path (schur.hip): interface lists of a plan

// Workspace for up to Kcap frequencies of one plan.
struct Work {
  const dyson_plan* plan = nullptr;  // plan the buffers were sized for
  int Kcap = 0;
  size_t bytes = 0;                  // device bytes held
  std::vector<void*> allocs;
  double *d = nullptr, *gacc = nullptr, *xB = nullptr, *xH = nullptr, *r = nullptr, *z = nullptr,
         *p0 = nullptr, *p1 = nullptr, *s = nullptr, *rhs = nullptr, *R = nullptr, *Q = nullptr;
  void* fac[2] = {nullptr, nullptr};
  double* fac64 = nullptr;  // complex128 leaf factors written with the leaf diagonal
  int fac_g[2] = {-1000, -1000};
  double* partial = nullptr;
  double *hpart = nullptr, *h = nullptr;
  CocgState cst{};
  int *lz_stopped = nullptr, *lz_steps = nullptr, *lz_reorth = nullptr, *lz_armed = nullptr;
  double* Dl = nullptr;  // diagonal correction of the level being run
  // Lanczos on the Schur complement: step vectors v_j = p_j + B^{-1} E p_j, the
  // projected Hessenberg matrices (one per item) and the inversion's scratch
  double *Vb = nullptr, *Hm = nullptr, *gjC = nullptr, *gjR = nullptr, *gjQ = nullptr;
  int* f1mask = nullptr;  // skip array of the fresh-direction continuation
  int *klist = nullptr, *kalive = nullptr, *d_kcount = nullptr;  // inner solves' open frequencies
  double *lz_alpha = nullptr, *lz_beta = nullptr, *lz_unorm2 = nullptr, *lz_umax2 = nullptr,
         *lz_scal = nullptr;
  int* d_count = nullptr;
  double* rho2 = nullptr;   // inner solves: r^T z of the last two iterations per item
  double* alph = nullptr;   // inner solves: alpha of the last even iteration per item
  double* partS = nullptr;  // inner solves: per-unit p^T A p
  double* stage_om = nullptr;  // [2*Kcap] staging of host-side frequencies
  std::vector<int> pred;    // predicted inner iterations per (level, graph) for polling
  // captured chunks of inner iterations, keyed by the launch arguments and
  // the first iteration; replayed on this Work's stream
  std::unordered_map<std::string, hipGraphExec_t> graphs;
  bool graphs_broken = false;  // a capture failed: direct launches from then on
  int* h_count = nullptr;   // pinned (h_static for a carved Work)
  // carved: the buffers are slices of a caller-provided region (the
  // allocation-free entry point); nothing is freed, no profiling events are
  // made and the correction levels run as one group on the call's stream
  bool carved = false;
  int h_static[4] = {0, 0, 0, 0};
  unsigned long long* d_prof = nullptr;
  unsigned long long* d_wprof = nullptr;  // [4][Kcap*nmax] per-item byte counts (profiling):
                                          // inner solves in [0,2), Lanczos in [2,4)
  uint64_t* d_fkey = nullptr;
  int* d_flag = nullptr;    // input validation flags
  double* d_err = nullptr;  // sampled error estimate
  Prof prof;
  // run statistics of the current call
  long long stat_inner = 0;
  int stat_inner_max = 0;
  int stat_restarts = 0;
  int stat_capped = 0;      // items stopped by the step cap before exhaustion
  dyson_status pending = DYSON_OK;
  int kq = 1;               // Lanczos steps the basis Q can hold (Q has kq + 1 vectors)
  // correction levels run concurrently: groups 1.. of the plan's level
  // groups run in these workspaces on their own streams (group 0 runs here)
  std::vector<std::unique_ptr<Work>> sub;
  std::vector<hipStream_t> sub_stream;
  hipEvent_t ev = nullptr;
};

}  // namespace dyson

struct dyson_ctx {
  int device = 0;
  size_t budget = 0;           // serving: device bytes the request slots may hold
  bool has_alloc = false;
  dyson_allocator alloc{};
  std::mutex server_mu;
  std::shared_ptr<dyson::Server> server;  // started by the first dyson_submit
  int slots = 3;
  int max_batch_freqs = 256;
  std::atomic<int> live_plans{0};
  ~dyson_ctx();  // stops the server (serve.cpp)
};

struct dyson_plan {
  dyson_ctx* ctx = nullptr;
  dyson::HostPlan hp;
  dyson::TileGeom geom{};
  int* d_nbr = nullptr;
  uint8_t* d_kind = nullptr;
  uint8_t* d_depth = nullptr;
  int* d_site_of = nullptr;
  int* d_pos_of = nullptr;
  std::vector<dyson::DevLevel> lv;
  int kcap = 1;     // largest Lanczos step cap + 1 (basis vectors)
  int nmax = 1;     // most domains on one level
  int nimax = 0;    // most tiles holding one level's interface sites (compact basis)
  int hstride = 1;
  std::vector<int> check_pos;  // tile positions of the sampled error check
  dyson::Work main;  // workspace of the blocking entry points
  dyson::Work carved;  // slices of the device's scratch array (dyson_solve_noalloc)
  std::shared_ptr<dyson::SchurData> schur;  // built by the first dyson_solve_schur
  std::atomic<int> live_requests{0};
};

namespace dyson {

// One contiguous run of frequencies of a batch: K rows of the caller's (or a
// staging) [K][N] arrays.  V is [N]; omega [K] Matsubara w_k (zmode 0) or
// [K] complex energies z_k (zmode 1); sigma and G [K][N] complex.
struct Slice {
  int K;
  const double* V;
  const double* omega;
  const double* sigma;
  double* G;
  int zmode;
};

// Correction levels per concurrent group: group 0 holds the level with the
// longest Lanczos run; within a group levels run bottom-up.
std::vector<std::vector<int>> level_groups(const dyson_plan* p);

// Device bytes a Work for K frequencies of the plan holds (with its groups).
size_t work_bytes(const dyson_plan* p, int K);
// Device bytes a carved Work (one level group) for K frequencies needs.
size_t carved_bytes(const dyson_plan* p, int K);
// Points every buffer of *w at consecutive 256-byte aligned slices of
// [base, base + cap) for K frequencies; DYSON_EINVAL if they do not fit.
dyson_status carve_work(const dyson_plan* p, Work* w, int K, char* base, size_t cap);
// Allocation-free path (noalloc.hip): records the device address of the
// device's scratch array; called once per device by dyson_create.
dyson_status noalloc_init(int device);
dyson_status ensure_work(const dyson_plan* p, Work* w, int K, hipStream_t s);
void free_work(Work* w, hipStream_t s);

// eq. (1) input checks on the device (w_k > 0, finite values,
// Im(i w_k - Sigma_i) > 0) for each slice; uses w->d_flag.
dyson_status validate_slices(const dyson_plan* p, Work* w, const Slice* sl, int n, hipStream_t s);

// Whole hot path for the concatenation of n slices (sum of K <= w->Kcap).
// `abort` is polled between correction levels; when it returns true the
// solve stops and returns DYSON_ECANCELLED.
dyson_status run_solve(dyson_plan* p, Work* w, const Slice* sl, int n, hipStream_t s,
                       dyson_report* rep, const std::function<bool()>& abort);

// Device memory through the context's allocator (hipMalloc without one).
void* ctx_alloc(const dyson_ctx* c, size_t bytes, hipStream_t s);
void ctx_free(const dyson_ctx* c, void* ptr, hipStream_t s);

// Frees the idle serving workspaces sized for plan p (before p is destroyed).
void serve_forget_plan(dyson_ctx* c, const dyson_plan* p);

}  // namespace dyson
