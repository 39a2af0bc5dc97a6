// Device-side argument blocks and kernel launchers (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dyson {

// Read-only geometry of a plan on the device (tile-major layout).
struct TileGeom {
  int T, S, sx, sy, N;   // sy block rows (slices) of sx sites per tile
  double t;
  const int* nbr;        // [T*6]: -x, +x, -y, +y, -z, +z
  const uint8_t* kind;   // [T*S] 0 pad, 1 leaf, 2 separator
  const uint8_t* depth;  // [T*S]
  const int* site_of;    // [T*S] natural index or -1
  const int* pos_of;     // [N]
  int edge;              // tile edge s (tile = s^dim sites)
  int dim;               // lattice dimension 1..3
  unsigned edge_magic;   // floor(2^32 / s) + 1: v / s = mulhi(v, edge_magic) for v < 2^16
};

// Per-item scalars of the inner COCG solves (item = k * n_nodes + node).
struct CocgState {
  int* done;       // 0 open, 1 closed at the start, else the mark of the closing launch
  int* iters;
  double* bn2;     // |b|^2
};

struct CocgLaunch {
  TileGeom G;
  int K;
  int g;                 // graph level: sites with depth >= g (and leaves) are active
  const int* tile_node;  // [T] domain of the tile at the Lanczos level
  int n_nodes;
  const int* item_skip;  // Lanczos "stopped" flags or null
  CocgState st;
  const double* d;
  double *x, *r, *z, *p_old, *p_new, *s;
  const void* fac;       // tile factors for graph g
  bool fp32;             // factors stored as complex64
  bool fp16;             // factors stored as complex32 (two FP16 halves)
  unsigned long long* wctr;  // profiling: [2][n_items] algorithmic bytes (update,
                             // stencil) booked by each item's lead wave, or null
  const int* tlo;        // [n_nodes] tile range of each domain
  const int* thi;
  int n_items;           // K * n_nodes
  double* partS;         // [K*T] complex: p^T A p per unit
  double* partU;         // [K*T*2] complex: r^T z and |r|^2 per unit
  double* rho2;          // [2][n_items] complex: r^T z of the last two iterations
  double* alph;          // [n_items] complex: alpha of the last even iteration (x is
                         // updated every other iteration, alpha_{i-1} p_{i-1} + alpha_i p_i)
  double tol2;           // squared relative residual target
  int flush;             // final stencil launch: close every open item
  const int* klist;      // frequencies with an open item (compacted), or null: every
                         // frequency; the stencil and update launches map their units
                         // through it, and the units past its length leave at once
  const int* kcount;     // [1] length of klist
  int* kalive;           // [K] stamp of the last launch after which frequency k still
                         // had an open item (1: the initial check, it + 2: stencil it)
};

struct LzArgs {
  TileGeom G;
  int level;
  const int* tile_node;
  int n_nodes;
  uint64_t seed;
  const uint64_t* fkey;  // [K] identity of frequency k (bits of w_k), keys the start vectors
  int* stopped;     // 0 open, 1 exhausted, 2 step cap, 3 breakdown, 4 done earlier
  int* steps;
  double* alpha;    // complex
  double* beta;     // complex: beta_j coupling q_{j-1}, q_j
  double* unorm2;   // |u|^2 of the current step
  double* umax2;    // running max of |u|^2 over the item's steps
  double* scal;     // complex
  double* partial;  // [K*T*2] complex
  double* hpart;    // [K*T*hstride] complex
  double* h;        // [K*n_nodes*hstride] complex
  int hstride;
  const int* tlo;   // [n_nodes] tile range of each domain (into tlist when it is set)
  const int* thi;
  const int* tlist; // tiles the Lanczos vectors live on, grouped by domain, or null
                    // (every tile of the level); the vector kernels run on these only
  int n_tlist;
  int qcompact;     // 1: the basis vectors and the residual are stored on the listed
                    // tiles only ([K][n_tlist][S]; other vectors keep [K][T][S])
  const int* tpos;  // [T] position of a tile in tlist, -1 if not listed (qcompact)
  int n_items;
  unsigned long long* wctr;  // profiling: [2][n_items] algorithmic bytes (CGS update,
                             // CGS products) booked by each item's lead block, or null
  int* reorth;      // [n_items] 1 if the second Gram-Schmidt pass runs for the item
  int* armed;       // [n_items] 1 after a step whose residual passed the L2 stop test:
                    // the next step confirms exhaustion (|X q| at the noise level)
  int iface;        // 1: Lanczos on the Schur complement (exactly m steps per item)
};

// Zeroes `bytes` bytes (a multiple of 4) at device address p on stream s.
void launch_zero(void* p, size_t bytes, hipStream_t s);
void launch_to_tile(const TileGeom& G, int K, const double* nat, double* tile, double fill_re,
                    hipStream_t s);
void launch_from_tile(const TileGeom& G, int K, const double* tile, double* nat, hipStream_t s);
// omega: w_k [K] (zmode 0, z_k = i w_k) or complex z_k [K] (zmode 1)
void launch_assemble(const TileGeom& G, int K, double mu, const double* V, const double* omega,
                     int zmode, const double* sigma, double* d, hipStream_t s);
// eq. (1) input checks, OR-ed into *flag: 1 non-finite V, 2 Im z_k <= 0 or
// non-finite z_k, 4 non-finite Sigma, 8 Im(z_k - Sigma_i) <= 0.
// With min_im > 0 also 16: Im(z_k - Sigma_i) < min_im (complex32 factors need
// their entries, bounded by 1 / min Im H_ii, inside the FP16 range).
void launch_validate(int N, int K, const double* V, const double* omega, int zmode,
                     const double* sigma, double min_im, int* flag, hipStream_t s);
// Tile block factors of graph g (complex128 / complex64 / complex32 storage).
void launch_factor(const TileGeom& G, int K, int g, const int* tile_node, const double* d,
                   void* fac, bool fp32, bool fp16, hipStream_t s);
// Leaf factors in complex128 (fac64) and the exact diagonal of every leaf block.
void launch_factor_diag(const TileGeom& G, int K, const double* d, double* fac64, double* gdiag,
                        hipStream_t s);

void launch_cocg_init(const CocgLaunch& L, const double* b, hipStream_t s);
void launch_cocg_stencil(const CocgLaunch& L, int it, hipStream_t s);
void launch_cocg_compact(const CocgLaunch& L, int stamp, int* klist, int* kcount, hipStream_t s);
void launch_cocg_check(const CocgLaunch& L, int it, int* open, hipStream_t s);
void launch_prof_collect(unsigned long long* per_item, int n, int classes, int first_class,
                         unsigned long long* tot, hipStream_t s);
void launch_cocg_update(const CocgLaunch& L, int it, hipStream_t s);
void launch_count_open(const int* done, int n, int* out, hipStream_t s);

void launch_freq_keys(const double* omega, int zmode, int K, uint64_t* fkey, hipStream_t s);
void launch_lz_random(const LzArgs& a, int K, double* q, uint64_t salt, hipStream_t s,
                      int real_only = 0);
void launch_lz_scale(const LzArgs& a, int K, double* q, hipStream_t s);
void launch_lz_defect(const LzArgs& a, int K, const double* q, const double* w, double* b,
                      hipStream_t s);
void launch_lz_alpha(const LzArgs& a, int K, const double* q, const double* u, hipStream_t s);
void launch_lz_recur(const LzArgs& a, int K, const double* q, const double* qprev, const double* u,
                     double* r, double* D, hipStream_t s);
// Gram-Schmidt pass `pass` (0: always; 1: only items whose reorth flag is set)
void launch_cgs_dot(const LzArgs& a, int K, const double* Q, size_t qstride, int nvec,
                    const double* r, int pass, hipStream_t s);
void launch_cgs_reduce(const LzArgs& a, int K, const int* tlo, const int* thi, int nvec, int pass,
                       hipStream_t s);
void launch_cgs_update(const LzArgs& a, int K, const double* Q, size_t qstride, int nvec, double* r,
                       double* D, int pass, hipStream_t s);
// After pass 0: reorth[item] = |r'|^2 < eta2 |r|^2 (the pass removed a large part of r)
void launch_cgs_decide(const LzArgs& a, int K, const int* tlo, const int* thi, int nvec,
                       double eta2, hipStream_t s);
void launch_lz_norms(const LzArgs& a, int K, const double* r, hipStream_t s);
void launch_lz_next(const LzArgs& a, int K, const double* r, double* qn, hipStream_t s);
// force (op 2): declare every open item broken down at this step (test hook)
void launch_lz_scalars(const LzArgs& a, int K, const int* tlo, const int* thi, const int* mcap,
                       int op, int j, double tol, double brk, int force, hipStream_t s);
void launch_lz_reopen(const LzArgs& a, int K, double* D, hipStream_t s);
// Lanczos on the Schur complement (iface.hip)
void launch_f1_rhs(const LzArgs& a, int K, const double* p, double* rhs, hipStream_t s);
void launch_f1_smat(const LzArgs& a, int K, const double* d, const double* p, const double* u,
                    double* sv, double* v, hipStream_t s);
void launch_f1_hcol(const LzArgs& a, double* Hm, int mm, int j, int op, hipStream_t s);
void launch_f1_mask(const LzArgs& a, int* mask, hipStream_t s);
void launch_f1_settle(const LzArgs& a, hipStream_t s);
void launch_f1_hzero(const LzArgs& a, double* Hm, int mm, hipStream_t s);
void launch_f1_hpad(const LzArgs& a, double* Hm, int mm, hipStream_t s);
void launch_f1_diag(const LzArgs& a, int K, const double* Vb, size_t qstride, const double* Minv,
                    int mm, double* D, hipStream_t s);
// In-place inverse of `batch` m x m complex matrices (schur.hip); scratch Cb
// [batch][m][32], Rx [batch][32][m], Qb [batch][32][32] complex.
void launch_gj_invert(double* A, int m, int batch, double* Cb, double* Rx, double* Qb,
                      hipStream_t s);
void launch_add_into(const LzArgs& a, int K, const double* D, double* G, hipStream_t s);
// Sampled check: b = e_pos in every frequency row; err = max(err, max_k |x - g| / |x|) at pos.
void launch_unit_vector(const TileGeom& G, int K, int pos, double* b, hipStream_t s);
void launch_sample_err(const TileGeom& G, int K, int pos, const double* x, const double* g,
                       double* err, hipStream_t s);

}  // namespace dyson
