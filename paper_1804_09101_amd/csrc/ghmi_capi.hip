// C interface (include/ghmi.h): context, domain setup, operator cache,
// GEMM tile lists with autotuned tile shape, and the RHS / RK3 / constraint
// drivers that queue the kernels of ghmi_kernels.hip on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "ghmi.h"
#include "ghmi_internal.h"
#include "ghmi_setup.h"
#include "ghmi_tensor_filter.h"

#include <mutex>

// Device scratch of gh_constraints_static: one array per GPU, held until the
// process ends.  Host code never uses this name as an address; it uses the
// per-device pointer that hipGetSymbolAddress returns (scratch_ptr below).
static __device__ __align__(256) double scratch[GH_STATIC_SCRATCH_DOUBLES];

namespace {

// Device address of `scratch` on each GPU, looked up once per device (with that
// device current) by gh_create.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

int lookup_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return GH_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[device]) return GH_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GH_ERR_DEVICE;
  g_scratch_ptr[device] = static_cast<double*>(p);
  return GH_OK;
}

// The GEMM work of one operation over the whole domain: groups of consecutive
// shells sharing an angular operator, cut into tiles of one tile shape.
struct GemmPlan {
  int shape = 0;
  int order = 0;                          // tile order, see build_tiles
  std::vector<GemmGroup> groups;          // host copy (operator pointers resolved)
  GemmGroup* d_full = nullptr;            // device copy of groups
  GemmGroup* d_groups = nullptr;          // groups of the main launch (d_full, or their leading rows)
  GemmTile* d_tiles = nullptr;
  int n_tiles = 0;
  // split plan: the trailing rows that would start one more round of tiles
  // on a few CUs go to a second launch of smaller tiles over K chunks
  // (partial products into d_work), then a chunk-ordered sum into C
  int tail_shape = -1, tail_order = 0, tail_chunks = 0;
  GemmGroup* d_tgroups = nullptr;
  GemmTile* d_ttiles = nullptr;
  int n_ttiles = 0;
  int tail_rows = 0, tail_cols = 0, tail_ldc = 0;
  long long tail_c_off = 0;
  double* d_work = nullptr;
};

}  // namespace

struct gh_ctx {
  int device = 0;
  int n_cu = 256;                // compute units of the device (tile rounds of the GEMM plans)
  hipStream_t stream = nullptr;
  std::string err = "";

  // domain
  int n_inst = 0, n_shells = 0;
  std::vector<gh_shell> shells;
  std::vector<long long> offs;   // n_shells + 1
  long long P = 0;
  int max_S = 0;
  int filter_kind = 0;
  double filt[3] = {0, 0, 0};
  bool have_domain = false, have_bg = false, have_gamma = false, have_dt = false;

  // tables
  std::vector<ShellDev> h_sh;
  std::vector<PtBlock> h_blk;
  ShellDev* d_sh = nullptr;
  PtBlock* d_blk = nullptr;
  int n_blk = 0;
  PtBlock* d_cblk = nullptr;   // column blocks (shell, first angular point) for the radial kernel
  PtBlock* d_fblk = nullptr;   // point blocks covering both faces of every interface
  int n_fblk = 0;
  int n_cblk = 0;
  int maxr = 0;                // register-array size of the column radial kernel (0: point form)
  double *d_dtab = nullptr, *d_angtab = nullptr, *d_radtab = nullptr, *d_bctab = nullptr;
  // interface projection from the state (gh_set_interface 1): its own table,
  // rebuilt from the state before every boundary treatment, and scratch for
  // the excision speeds the table kernel also writes
  int iface_mode = 0, bc_total = 0;
  int outer_mode = 0;                  // gh_set_outer_bc: 0 Dirichlet, 1 constraint-preserving
  double *d_bctab_s = nullptr, *d_exscr = nullptr;
  std::map<int, double*> d_angop;   // per L: [S][2S], B operand (Theta^T | Phi^T)
  std::map<int, double*> d_filtop;  // per L: [S][S], B operand F^T
  std::map<int, double*> d_angopT;  // per L: [2S][S], B operand (Theta ; Phi) of the transposed derivative
  std::map<int, double*> d_filtopT; // per L: [S][S], B operand F of the transposed filter
  GemmPlan deriv, filter, derivT, filterT;
  int* d_shell_range = nullptr;     // per instance: first and one-past-last shell

  // adjoint work space (allocated on first use)
  bool have_adj = false;
  double *d_Lb = nullptr, *d_dRb = nullptr, *d_dAb = nullptr, *d_T = nullptr;
  double *d_u1 = nullptr, *d_u2 = nullptr, *d_lam3 = nullptr, *d_mu1 = nullptr, *d_mu2 = nullptr;
  double *d_gpart = nullptr, *d_bcg = nullptr;
  double* d_vacc = nullptr;          // [12][P]: geometry and gamma cotangents between the two reverse pointwise passes
  double *d_C = nullptr, *d_norm = nullptr;   // constraint values and norms for gh_constraints_vjp

  // Dormand-Prince work space (allocated on first use): seven stage
  // derivatives, the stage state, the fifth-order solution, its filtered copy,
  // per-instance flags and value counts
  // transform path of the angular operators (gh_set_angular 1, built on first use)
  int ang_method = 0;
  bool deriv_tr = false, filt_tr = false;    // effective choices (method 2 picks each by timing)
  bool have_tr = false;
  double *d_ktab = nullptr, *d_X = nullptr;
  PtBlock* d_tblk = nullptr;                 // blocks of the theta step: 16 rows x 256 (node, column) pairs
  int n_tblk = 0, tr_nmax = 0;
  // the matrix-core theta step for shells with n = L + 1 in {16, 32, 48, 64}:
  // the transposed kernel table and the work items per n
  double* d_ktabT = nullptr;
  ThetaItem* d_titem[4] = {nullptr, nullptr, nullptr, nullptr};
  int n_titem[4] = {0, 0, 0, 0};
  std::map<int, double*> d_fana, d_fsyn;    // per L: Fourier analysis [2n][2n] and synthesis (its transpose)
  GemmPlan tr_ana, tr_syn, tr_fsyn;

  // tensor-coupled filter (filter_kind 2, 3): PhysToSpec GEMM into the
  // coefficient array X (per shell [field][radius][nsp], nsp = (L+1)^2 rounded
  // up to even so that rows stay 16-byte aligned), coupling into Y,
  // SpecToPhys GEMM; the adjoint uses the transposed matrices
  std::map<int, double*> d_anaT, d_synT, d_syn, d_ana;   // per L: B operands [S][nsp], [ns][S], [S][nsp], [ns][S]
  double *d_tfx = nullptr, *d_tfy = nullptr;
  double* d_legtab = nullptr;                // per L: Legendre analysis and synthesis tables (transform form)
  PtBlock *d_lg_ablk = nullptr, *d_lg_sblk = nullptr;
  int n_lg_ablk = 0, n_lg_sblk = 0;
  GemmPlan tf_p2s, tf_s2p, tf_p2sT, tf_s2pT;
  TfItem* d_tf_items = nullptr;
  TfSeg* d_tf_segs = nullptr;
  TfCol* d_tf_cols = nullptr;
  long long *d_tf_soff = nullptr, *d_tfT_soff = nullptr;   // sliced-ELL of F and of F^T
  int *d_tf_swid = nullptr, *d_tfT_swid = nullptr;
  int *d_tf_perm = nullptr, *d_tfT_perm = nullptr;
  int *d_tf_lidx = nullptr, *d_tfT_lidx = nullptr;
  double *d_tf_val = nullptr, *d_tfT_val = nullptr;
  int n_tf_items[3] = {0, 0, 0};
  long long tf_nnz = 0;

  bool have_dp5 = false;
  double *d_dpk = nullptr, *d_dpy = nullptr, *d_dpu5 = nullptr, *d_dpf = nullptr, *d_dpnval = nullptr;
  int *d_dprej = nullptr, *d_dpacc = nullptr;

  // reductions
  int* d_inst_range = nullptr;
  double *d_wsum = nullptr, *d_partial = nullptr;

  // work space and state
  double *d_dR = nullptr, *d_dA = nullptr, *d_W = nullptr, *d_ua = nullptr, *d_ub = nullptr;
  double *d_H = nullptr, *d_dH = nullptr;
  double *d_gamma = nullptr, *d_dt = nullptr;
  std::vector<void*> allocs;

  // step graphs (gh_set_graph): one captured SSP-RK3 step per state pointer
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  const double* graph_u = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;

  // kernel timing (gh_set_timing): every kind, or (timing_only >= 0) one kind
  bool timing = false;
  int timing_only = -1;
  struct Rec { hipEvent_t a, b; int kind; };
  std::vector<Rec> recs;
};

namespace {

int fail(gh_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                            \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(ctx, GH_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Bracket one launch with events when timing is on.
struct Timed {
  gh_ctx* c;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(gh_ctx* c_, int k) : c(c_), kind(k) {
    if (c->timing && (c->timing_only < 0 || c->timing_only == k) && hipEventCreate(&a) == hipSuccess &&
        hipEventCreate(&b) == hipSuccess)
      (void)hipEventRecord(a, c->stream);
  }
  ~Timed() {
    if (a && b) {
      (void)hipEventRecord(b, c->stream);
      c->recs.push_back(gh_ctx::Rec{a, b, kind});
    }
  }
};

// The reverse pass's stage combinations, timed as kind 5 (the forward stage
// update is timed with the boundary treatment it includes, kind 4).
#define LINCOMB(expr)          \
  do {                         \
    Timed t_(c, 5);            \
    HIPCHK(c, expr);           \
  } while (0)

void clear_timing(gh_ctx* c) {
  for (auto& r : c->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  c->recs.clear();
}

void drop_graph(gh_ctx* c) {
  if (c->cap_stream) (void)hipStreamSynchronize(c->cap_stream);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
  c->graph_u = nullptr;
}

void free_domain(gh_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  clear_timing(c);
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  c->d_angop.clear();
  c->d_filtop.clear();
  c->d_angopT.clear();
  c->d_filtopT.clear();
  c->deriv = GemmPlan();
  c->filter = GemmPlan();
  c->derivT = GemmPlan();
  c->filterT = GemmPlan();
  c->d_shell_range = nullptr;
  c->have_adj = false;
  c->d_Lb = c->d_dRb = c->d_dAb = c->d_T = nullptr;
  c->d_u1 = c->d_u2 = c->d_lam3 = c->d_mu1 = c->d_mu2 = nullptr;
  c->d_gpart = c->d_bcg = nullptr;
  c->d_vacc = nullptr;
  c->d_C = c->d_norm = nullptr;
  c->ang_method = 0;
  c->deriv_tr = c->filt_tr = false;
  c->have_tr = false;
  c->d_ktab = c->d_X = nullptr;
  c->d_tblk = nullptr;
  c->d_ktabT = nullptr;
  for (int k = 0; k < 4; ++k) {
    c->d_titem[k] = nullptr;
    c->n_titem[k] = 0;
  }
  c->n_tblk = c->tr_nmax = 0;
  c->d_fana.clear();
  c->d_fsyn.clear();
  c->tr_ana = GemmPlan();
  c->tr_syn = GemmPlan();
  c->tr_fsyn = GemmPlan();
  c->d_anaT.clear();
  c->d_synT.clear();
  c->d_syn.clear();
  c->d_ana.clear();
  c->tf_p2s = GemmPlan();
  c->tf_s2p = GemmPlan();
  c->tf_p2sT = GemmPlan();
  c->tf_s2pT = GemmPlan();
  c->d_tfx = c->d_tfy = nullptr;
  c->d_legtab = nullptr;
  c->d_lg_ablk = c->d_lg_sblk = nullptr;
  c->n_lg_ablk = c->n_lg_sblk = 0;
  c->d_tf_items = nullptr;
  c->d_tf_segs = nullptr;
  c->d_tf_cols = nullptr;
  c->d_tf_soff = c->d_tfT_soff = nullptr;
  c->d_tf_swid = c->d_tfT_swid = nullptr;
  c->d_tf_perm = c->d_tfT_perm = nullptr;
  c->d_tf_lidx = c->d_tfT_lidx = nullptr;
  c->d_tf_val = c->d_tfT_val = nullptr;
  c->n_tf_items[0] = c->n_tf_items[1] = c->n_tf_items[2] = 0;
  c->tf_nnz = 0;
  c->have_dp5 = false;
  c->d_dpk = c->d_dpy = c->d_dpu5 = c->d_dpf = c->d_dpnval = nullptr;
  c->d_dprej = c->d_dpacc = nullptr;
  c->d_sh = nullptr; c->d_blk = nullptr; c->d_cblk = nullptr; c->d_fblk = nullptr;
  c->d_dtab = c->d_angtab = c->d_radtab = c->d_bctab = nullptr;
  c->iface_mode = c->bc_total = 0;
  c->outer_mode = 0;
  c->d_bctab_s = c->d_exscr = nullptr;
  c->d_inst_range = nullptr; c->d_wsum = c->d_partial = nullptr;
  c->d_dR = c->d_dA = c->d_W = c->d_ua = c->d_ub = nullptr;
  c->d_H = c->d_dH = nullptr;
  c->d_gamma = c->d_dt = nullptr;
  c->have_domain = c->have_bg = c->have_gamma = c->have_dt = false;
}

template <class T>
int dalloc(gh_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(c, GH_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  c->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return GH_OK;
}

// Free one allocation of the context early (the others go in free_domain).
template <class T>
void dfree(gh_ctx* c, T*& p) {
  if (!p) return;
  auto it = std::find(c->allocs.begin(), c->allocs.end(), static_cast<void*>(p));
  if (it != c->allocs.end()) {
    (void)hipFree(p);
    c->allocs.erase(it);
  }
  p = nullptr;
}

template <class T>
int upload(gh_ctx* c, T** p, const std::vector<T>& h) {
  int rc = dalloc(c, p, h.size());
  if (rc) return rc;
  if (!h.empty()) HIPCHK(c, hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return GH_OK;
}

// Free the device tile lists and split work space of a plan (its groups stay),
// so that re-planning (tuning trials, pinning) does not accumulate buffers.
void plan_release(gh_ctx* c, GemmPlan& pl) {
  if (!pl.d_tiles && !pl.d_tgroups && !pl.d_ttiles && !pl.d_work) return;
  // queued launches may still read the lists
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->cap_stream) (void)hipStreamSynchronize(c->cap_stream);
  dfree(c, pl.d_tiles);
  if (pl.d_groups != pl.d_full) dfree(c, pl.d_groups);
  pl.d_groups = nullptr;
  dfree(c, pl.d_tgroups);
  dfree(c, pl.d_ttiles);
  dfree(c, pl.d_work);
  pl.n_tiles = pl.n_ttiles = 0;
  pl.tail_shape = -1;
  pl.tail_chunks = 0;
}

// Build the tile list of a plan for one kernel variant and tile order and upload it.
int plan_upload(gh_ctx* c, GemmPlan& pl, int shape, int order) {
  plan_release(c, pl);
  std::vector<GemmTile> tiles = ghk::build_tiles(pl.groups, shape, order);
  pl.shape = shape;
  pl.order = order;
  pl.n_tiles = int(tiles.size());
  pl.tail_shape = -1;
  pl.n_ttiles = 0;
  int rc;
  if (!pl.d_full) {
    if ((rc = upload(c, &pl.d_full, pl.groups))) return rc;
  }
  pl.d_groups = pl.d_full;
  if ((rc = upload(c, &pl.d_tiles, tiles))) return rc;
  return GH_OK;
}

// Rows of a plan's groups split for whole rounds of tiles: with `shape`, the
// main launch keeps n_cu * floor(tiles / n_cu) tiles (whole row tiles, peeled
// from the end of the last groups) and the peeled rows form the tail groups.
// False when the tile count is already a multiple of n_cu or below it.
bool split_rows(const std::vector<GemmGroup>& gs, int shape, int n_cu, std::vector<GemmGroup>& mainv,
                std::vector<GemmGroup>& tailv) {
  int bm, bn;
  ghk::tile_dims(shape, &bm, &bn);
  long long total = 0;
  for (const auto& g : gs) total += (long long)((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn);
  const long long target = (long long)n_cu * (total / n_cu);
  if (target == 0 || target == total) return false;
  mainv = gs;
  tailv.clear();
  long long cur = total;
  for (int gi = int(gs.size()) - 1; gi >= 0 && cur > target; --gi) {
    GemmGroup& g = mainv[gi];
    const int nt = (g.N + bn - 1) / bn;
    int mt = (g.M + bm - 1) / bm;
    while (mt > 0 && cur > target) {
      --mt;
      cur -= nt;
    }
    const int keep = std::min(g.M, mt * bm);
    if (keep == g.M) continue;
    GemmGroup t = gs[gi];
    t.a_off += (long long)keep * t.lda;
    t.c_off += (long long)keep * t.ldc;
    t.M = g.M - keep;
    tailv.insert(tailv.begin(), t);
    g.M = keep;
  }
  return !tailv.empty();
}

// Upload a split plan: the main rows with (shape, order); the tail rows (one
// group) cut into `chunks` K ranges, each a group writing its partial product
// into the plan's work space, with (tail_shape, order 1).
int plan_upload_split(gh_ctx* c, GemmPlan& pl, const std::vector<GemmGroup>& mainv, const GemmGroup& tail,
                      int shape, int order, int tail_shape, int chunks) {
  const int kc = ((tail.K + chunks - 1) / chunks + 15) / 16 * 16;
  std::vector<GemmGroup> kv;
  for (int k0 = 0; k0 < tail.K; k0 += kc) {
    GemmGroup g = tail;
    g.a_off = tail.a_off + k0;
    g.B = tail.B + (long long)k0 * tail.ldb;
    g.K = std::min(kc, tail.K - k0);
    g.c_off = (long long)kv.size() * tail.M * tail.N;
    g.ldc = tail.N;
    kv.push_back(g);
  }
  plan_release(c, pl);
  std::vector<GemmTile> tiles = ghk::build_tiles(mainv, shape, order);
  std::vector<GemmTile> ttiles = ghk::build_tiles(kv, tail_shape, 1);
  int rc;
  if ((rc = upload(c, &pl.d_groups, mainv))) return rc;
  if ((rc = upload(c, &pl.d_tiles, tiles))) return rc;
  if ((rc = upload(c, &pl.d_tgroups, kv))) return rc;
  if ((rc = upload(c, &pl.d_ttiles, ttiles))) return rc;
  if ((rc = dalloc(c, &pl.d_work, kv.size() * size_t(tail.M) * tail.N))) return rc;
  pl.shape = shape;
  pl.order = order;
  pl.n_tiles = int(tiles.size());
  pl.tail_shape = tail_shape;
  pl.tail_order = 1;
  pl.tail_chunks = int(kv.size());
  pl.n_ttiles = int(ttiles.size());
  pl.tail_rows = tail.M;
  pl.tail_cols = tail.N;
  pl.tail_ldc = tail.ldc;
  pl.tail_c_off = tail.c_off;
  return GH_OK;
}

// One grouped GEMM of a plan: the main tile list; for a split plan then the
// tail's partial products (a role that overwrites) and their sum into C
// (added to C for role 2, C += A B).
hipError_t launch_plan(const GemmPlan& pl, const double* src, double* dst, hipStream_t st, int role) {
  hipError_t e = ghk::gemm(pl.shape, pl.d_tiles, pl.n_tiles, pl.d_groups, src, dst, st, role);
  if (e != hipSuccess || pl.n_ttiles == 0) return e;
  e = ghk::gemm(pl.tail_shape, pl.d_ttiles, pl.n_ttiles, pl.d_tgroups, src, pl.d_work, st, role == 2 ? 0 : role);
  if (e != hipSuccess) return e;
  return ghk::sum_chunks(pl.d_work, pl.tail_chunks, pl.tail_rows, pl.tail_cols, dst + pl.tail_c_off, pl.tail_ldc,
                         role == 2, st);
}

// Five launches of a plan after one untimed, in ms.
int time_plan(gh_ctx* c, const GemmPlan& pl, const double* src, double* dst, int role, hipEvent_t e0,
              hipEvent_t e1, float* ms) {
  HIPCHK(c, launch_plan(pl, src, dst, c->stream, role));
  HIPCHK(c, hipEventRecord(e0, c->stream));
  for (int it = 0; it < 5; ++it) HIPCHK(c, launch_plan(pl, src, dst, c->stream, role));
  HIPCHK(c, hipEventRecord(e1, c->stream));
  HIPCHK(c, hipEventSynchronize(e1));
  HIPCHK(c, hipEventElapsedTime(ms, e0, e1));
  return GH_OK;
}

// Time every (tile shape, tile order) on the plan (A = src, C = dst work
// space) and keep the fastest.  Of the fastest shape's orders, order 2 (blocks
// of 8 x 8 tiles per XCD) is kept when it is within 1% of the fastest: orders
// that time alike can move very different bytes (on the 20-shell derivative
// GEMM order 1 fetches twice what order 2 does, at the same speed), and
// closer timings flip from run to run.
int autotune(gh_ctx* c, GemmPlan& pl, const double* src, double* dst, int role) {
  float best = 1e30f;
  int best_shape = 0, best_order = 0;
  float t_order[ghk::NUM_TILE_SHAPES][ghk::NUM_TILE_ORDERS];
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  for (int sh = 0; sh < ghk::NUM_TILE_SHAPES; ++sh) {
    if (!ghk::shape_fits(sh, pl.groups)) continue;
    for (int order = 0; order < ghk::NUM_TILE_ORDERS; ++order) {
      int rc = plan_upload(c, pl, sh, order);
      if (rc) return rc;
      float ms = 0;
      if ((rc = time_plan(c, pl, src, dst, role, e0, e1, &ms))) return rc;
      t_order[sh][order] = ms;
      if (ms < best) {
        best = ms;
        best_shape = sh;
        best_order = order;
      }
    }
  }
  if (best_order != 2 && t_order[best_shape][2] <= 1.01f * best) {
    best_order = 2;
    best = t_order[best_shape][2];
  }
  // the fastest variant split for whole rounds of tiles, its tail rows in
  // smaller tiles of another variant; kept only when at least 1% faster than
  // one launch (closer timings flip from run to run)
  int best_tail = -1, best_chunks = 0;
  best *= 0.99f;
  std::vector<GemmGroup> mainv, tailv;
  if (split_rows(pl.groups, best_shape, c->n_cu, mainv, tailv) && tailv.size() == 1) {
    int bm, bn;
    ghk::tile_dims(best_shape, &bm, &bn);
    for (int ts = 0; ts < ghk::NUM_TILE_SHAPES; ++ts) {
      int tbm, tbn;
      ghk::tile_dims(ts, &tbm, &tbn);
      if (ts == best_shape || tbm * tbn >= bm * bn || !ghk::shape_fits(ts, tailv)) continue;
      for (int chunks = 2; chunks <= 8; chunks *= 2) {
        if (tailv[0].K < 16 * chunks) continue;
        int rc = plan_upload_split(c, pl, mainv, tailv[0], best_shape, best_order, ts, chunks);
        if (rc) return rc;
        float ms = 0;
        if ((rc = time_plan(c, pl, src, dst, role, e0, e1, &ms))) return rc;
        if (ms < best) {
          best = ms;
          best_tail = ts;
          best_chunks = chunks;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_tail >= 0)
    return plan_upload_split(c, pl, mainv, tailv[0], best_shape, best_order, best_tail, best_chunks);
  return plan_upload(c, pl, best_shape, best_order);
}

int check_ready(gh_ctx* c, bool need_dt) {
  if (!c) return GH_ERR_ARG;
  if (!c->have_domain) return fail(c, GH_ERR_ORDER, "gh_set_domain has not been called");
  if (!c->have_bg) return fail(c, GH_ERR_ORDER, "gh_set_background has not been called");
  if (!c->have_gamma) return fail(c, GH_ERR_ORDER, "gh_set_params has not been called");
  if (need_dt && !c->have_dt) return fail(c, GH_ERR_ORDER, "no time step set (gh_set_params dt)");
  return GH_OK;
}

int validate_shells(int n_inst, int n_shells, const gh_shell* s, std::string& why) {
  if (n_inst <= 0 || n_shells <= 0 || !s) { why = "need n_inst > 0, n_shells > 0, shells != NULL"; return GH_ERR_ARG; }
  for (int k = 0; k < n_shells; ++k) {
    if (s[k].n_r < 3 || s[k].n_r > 256 || s[k].L < 1 || s[k].L > 63) {
      why = "shell " + std::to_string(k) + ": need 3 <= n_r <= 256 and 1 <= L <= 63";
      return GH_ERR_ARG;
    }
    if (!(s[k].r_in > 0.0) || !(s[k].r_out > s[k].r_in) || !std::isfinite(s[k].r_out)) {
      why = "shell " + std::to_string(k) + ": need 0 < r_in < r_out";
      return GH_ERR_ARG;
    }
    if (s[k].instance < 0 || s[k].instance >= n_inst) {
      why = "shell " + std::to_string(k) + ": instance out of range";
      return GH_ERR_ARG;
    }
    if (k > 0) {
      if (s[k].instance < s[k - 1].instance) { why = "shells must be grouped by increasing instance"; return GH_ERR_SHAPE; }
      if (s[k].instance == s[k - 1].instance) {
        if (s[k].L != s[k - 1].L) { why = "adjacent shells of one instance must share L"; return GH_ERR_SHAPE; }
        if (s[k].r_in != s[k - 1].r_out) { why = "adjacent shells must satisfy r_out(k) == r_in(k+1)"; return GH_ERR_SHAPE; }
      } else if (s[k].instance != s[k - 1].instance + 1) {
        why = "every instance needs at least one shell"; return GH_ERR_SHAPE;
      }
    }
  }
  if (s[0].instance != 0 || s[n_shells - 1].instance != n_inst - 1) { why = "every instance needs at least one shell"; return GH_ERR_SHAPE; }
  return GH_OK;
}

// All derivative work of one RHS: the angular GEMM and the radial derivative.
// Radial (dR, [50] layout) and angular (dA, [100] layout) derivatives of u;
// into the context's work space unless targets are given.
// The theta step of the transform path (d_W -> d_X): the matrix-core kernel
// for shells with n a multiple of 16, the register kernel for the others.
int queue_theta(gh_ctx* c, int mode) {
  HIPCHK(c, ghk::ang_theta(c->tr_nmax, c->d_sh, c->d_tblk, c->n_tblk, c->d_ktab, c->d_W, c->d_X, mode, c->stream));
  for (int g = 0; g < 4; ++g)
    HIPCHK(c, ghk::ang_theta_mfma(16 * (g + 1), c->d_sh, c->d_titem[g], c->n_titem[g], c->d_ktabT, c->d_W, c->d_X,
                                  mode, c->stream));
  return GH_OK;
}

int queue_derivs(gh_ctx* c, const double* u, double* dR = nullptr, double* dA = nullptr) {
  if (!dR) dR = c->d_dR;
  if (!dA) dA = c->d_dA;
  if (c->deriv_tr) {
    // Fourier analysis into the RHS work space (free until the pointwise
    // kernel), theta kernels, synthesis into dA
    Timed t(c, 8);
    HIPCHK(c, launch_plan(c->tr_ana, u, c->d_W,
                        c->stream, 4));
    int rc;
    if ((rc = queue_theta(c, 0))) return rc;
    HIPCHK(c, launch_plan(c->tr_syn, c->d_X, dA,
                        c->stream, 5));
  } else {
    Timed t(c, 0);
    HIPCHK(c, launch_plan(c->deriv, u, dA, c->stream,
                        0));
  }
  {
    Timed t(c, 2);
    if (c->maxr)
      HIPCHK(c, ghk::radial_col(c->maxr, c->d_sh, c->d_cblk, c->n_cblk, c->d_dtab, u, dR, 0, 50, false, false,
                                c->stream));
    else
      HIPCHK(c, ghk::radial(c->d_sh, c->d_blk, c->n_blk, c->d_dtab, u, dR, 0, 50, false, false, c->stream));
  }
  return GH_OK;
}

// The tensor-coupled filter (or its transpose) of a whole state, src -> dst:
// PhysToSpec of every component, the component coupling, SpecToPhys.
int queue_tensor_filter(gh_ctx* c, const double* src, double* dst, bool transpose) {
  double* X = c->d_tfx;
  double* Y = c->d_tfy;
  const GemmPlan& p2s = transpose ? c->tf_p2sT : c->tf_p2s;
  const GemmPlan& s2p = transpose ? c->tf_s2pT : c->tf_s2p;
  const bool tr = c->filt_tr && !transpose;   // by transforms: Fourier GEMM + per-order Legendre steps
  if (tr) {
    HIPCHK(c, launch_plan(c->tr_ana, src, c->d_W,
                        c->stream, 4));
    HIPCHK(c, ghk::leg_analysis(c->d_sh, c->d_lg_ablk, c->n_lg_ablk, c->d_legtab, c->d_W, X, c->stream));
  } else {
    HIPCHK(c, launch_plan(p2s, src, X, c->stream, 6));
  }
  {
    Timed t(c, 9);
    HIPCHK(c, ghk::tensor_couple(c->d_tf_items, c->n_tf_items, c->d_tf_segs, c->d_tf_cols,
                                 transpose ? c->d_tfT_soff : c->d_tf_soff, transpose ? c->d_tfT_swid : c->d_tf_swid,
                                 transpose ? c->d_tfT_perm : c->d_tf_perm, transpose ? c->d_tfT_lidx : c->d_tf_lidx,
                                 transpose ? c->d_tfT_val : c->d_tf_val, X, Y, c->stream));
  }
  if (tr) {
    HIPCHK(c, ghk::leg_synthesis(c->d_sh, c->d_lg_sblk, c->n_lg_sblk, c->d_legtab, Y, c->d_W, c->stream));
    HIPCHK(c, launch_plan(c->tr_fsyn, c->d_W, dst,
                        c->stream, 5));
  } else {
    HIPCHK(c, launch_plan(s2p, Y, dst, c->stream, 7));
  }
  return GH_OK;
}

// The angular filter of a whole state, src -> dst (distinct); uses the RHS work
// space in the transform method and for the tensor-coupled filter.
int queue_filter(gh_ctx* c, const double* src, double* dst) {
  Timed t(c, 1);
  if (c->filter_kind >= 2) return queue_tensor_filter(c, src, dst, false);
  if (c->filt_tr) {
    HIPCHK(c, launch_plan(c->tr_ana, src, c->d_W,
                        c->stream, 4));
    int rc;
    if ((rc = queue_theta(c, 1))) return rc;
    HIPCHK(c, launch_plan(c->tr_fsyn, c->d_X, dst,
                        c->stream, 5));
  } else {
    HIPCHK(c, launch_plan(c->filter, src, dst,
                        c->stream, 1));
  }
  return GH_OK;
}

// The interface table the boundary treatment of d_t u(x) uses: the frozen
// one, or (gh_set_interface 1) one rebuilt from x now.
int interface_table(gh_ctx* c, const double* x, const double** tab) {
  if (!c->iface_mode) {
    *tab = c->d_bctab;
    return GH_OK;
  }
  HIPCHK(c, ghk::bc_setup(c->d_sh, c->n_shells, c->max_S, c->d_angtab, x, c->d_bctab_s, c->d_exscr, c->stream));
  *tab = c->d_bctab_s;
  return GH_OK;
}

int queue_rhs(gh_ctx* c, const double* u, double* out) {
  int rc = queue_derivs(c, u);
  if (rc) return rc;
  {
    Timed t(c, 3);
    HIPCHK(c, ghk::pointwise_rhs(c->d_sh, c->d_blk, c->n_blk, c->d_angtab, c->d_radtab, u, c->d_dR, c->d_dA,
                                 c->d_H, c->d_dH, c->d_gamma, out, c->stream));
  }
  {
    Timed t(c, 4);
    const double* tab = nullptr;
    if ((rc = interface_table(c, u, &tab))) return rc;
    if (c->outer_mode)
      HIPCHK(c, ghk::outer_cpbc(c->d_sh, c->n_shells, c->max_S, c->d_angtab, c->d_radtab, u, c->d_dR, c->d_dA,
                                c->d_gamma, out, c->stream));
    HIPCHK(c, ghk::boundary(c->d_sh, c->n_shells, c->max_S, tab, c->d_gamma, out, c->outer_mode, c->stream));
  }
  return GH_OK;
}

// One SSP-RK3 stage: out = c0 u0 + c1 (us + dt L(us)).  The pointwise kernel
// writes the stage value of every point off the treated faces straight to
// out, and the raw d_t u of the face points to the work space; the face
// kernel then applies the boundary treatment there and finishes the stage.
// With `keep` (150 P doubles) the derivatives of us are written there and kept.
int queue_stage(gh_ctx* c, double c0, const double* u0, double c1, const double* us, double* out,
                double* keep = nullptr) {
  double* dR = keep ? keep : c->d_dR;
  double* dA = keep ? keep + size_t(50) * c->P : c->d_dA;
  int rc = queue_derivs(c, us, dR, dA);
  if (rc) return rc;
  {
    Timed t(c, 3);
    HIPCHK(c, ghk::pointwise_stage(c->d_sh, c->d_blk, c->n_blk, c->d_angtab, c->d_radtab, us, dR, dA, c->d_H,
                                   c->d_dH, c->d_gamma, c->d_W, c->d_dt, c0, u0, c1, out, c->stream));
  }
  {
    Timed t(c, 4);
    const double* tab = nullptr;
    if ((rc = interface_table(c, us, &tab))) return rc;
    if (c->outer_mode)
      HIPCHK(c, ghk::outer_cpbc(c->d_sh, c->n_shells, c->max_S, c->d_angtab, c->d_radtab, us, dR, dA, c->d_gamma,
                                c->d_W, c->stream));
    HIPCHK(c, ghk::stage_faces(c->d_sh, c->n_shells, c->max_S, tab, c->d_gamma, c->d_dt, c0, u0, c1, us, c->d_W,
                               out, c->outer_mode, c->stream));
  }
  return GH_OK;
}

// One SSP-RK3 step (three stages, then the filter) in place on u.
int queue_step(gh_ctx* c, double* u) {
  int rc;
  const bool filt = c->filter_kind != 0;
  if ((rc = queue_stage(c, 0.0, nullptr, 1.0, u, c->d_ua))) return rc;
  if ((rc = queue_stage(c, 0.75, u, 0.25, c->d_ua, c->d_ub))) return rc;
  double* dst = filt ? c->d_ua : u;
  if ((rc = queue_stage(c, 1.0 / 3.0, u, 2.0 / 3.0, c->d_ub, dst))) return rc;
  if (filt)
    if ((rc = queue_filter(c, c->d_ua, u))) return rc;
  return GH_OK;
}

// Allocate the adjoint work space and choose tile shapes of the transposed GEMMs.
int ensure_adjoint(gh_ctx* c) {
  if (c->have_adj) return GH_OK;
  size_t F50 = size_t(50) * c->P;
  int rc;
  if ((rc = dalloc(c, &c->d_Lb, F50))) return rc;
  if ((rc = dalloc(c, &c->d_dRb, F50))) return rc;
  if ((rc = dalloc(c, &c->d_dAb, 2 * F50))) return rc;
  if ((rc = dalloc(c, &c->d_T, F50))) return rc;
  if ((rc = dalloc(c, &c->d_u1, F50))) return rc;
  if ((rc = dalloc(c, &c->d_u2, F50))) return rc;
  if ((rc = dalloc(c, &c->d_lam3, F50))) return rc;
  if ((rc = dalloc(c, &c->d_mu1, F50))) return rc;
  if ((rc = dalloc(c, &c->d_mu2, F50))) return rc;
  if ((rc = dalloc(c, &c->d_gpart, size_t(3) * c->n_blk))) return rc;
  if ((rc = dalloc(c, &c->d_vacc, size_t(12) * c->P))) return rc;
  if ((rc = dalloc(c, &c->d_bcg, size_t(c->n_shells) * c->max_S))) return rc;
  if ((rc = dalloc(c, &c->d_C, size_t(64) * c->P))) return rc;
  if ((rc = dalloc(c, &c->d_norm, size_t(c->n_inst)))) return rc;
  HIPCHK(c, ghk::fill_pattern(c->d_dAb, (long long)(2 * F50), c->stream));
  HIPCHK(c, ghk::fill_pattern(c->d_T, (long long)F50, c->stream));
  if ((rc = autotune(c, c->derivT, c->d_dAb, c->d_T, 2))) return rc;
  if (c->filter_kind == 1)
    if ((rc = autotune(c, c->filterT, c->d_T, c->d_Lb, 3))) return rc;
  if (c->filter_kind >= 2) {
    if ((rc = autotune(c, c->tf_p2sT, c->d_T, c->d_tfx, 6))) return rc;
    if ((rc = autotune(c, c->tf_s2pT, c->d_tfx, c->d_Lb, 7))) return rc;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->have_adj = true;
  return GH_OK;
}

// out = (d RHS / d u)^T mu at state x; adds coef * (use_dt ? dt : 1) * (dRHS/dgamma)^T mu
// to g (device [n_inst][3]) if g is not null.  Uses d_W, d_dA, d_dR, d_Lb, d_dRb, d_dAb.
// `kept`: derivatives of x saved by gh_step_stages (150 P doubles), else they
// are recomputed here.
int queue_rhs_vjp(gh_ctx* c, const double* x, const double* mu, double* out, double coef, int use_dt,
                  double* g, const double* kept = nullptr) {
  const double* dR = kept ? kept : c->d_dR;
  const double* dA = kept ? kept + size_t(50) * c->P : c->d_dA;
  if (!kept) {
    int rc = queue_derivs(c, x);
    if (rc) return rc;
  }
  // the transposed exchange needs the raw d_t u only on interface faces
  if (c->n_fblk)
    HIPCHK(c, ghk::pointwise_rhs(c->d_sh, c->d_fblk, c->n_fblk, c->d_angtab, c->d_radtab, x, dR, dA, c->d_H,
                                 c->d_dH, c->d_gamma, c->d_W, c->stream));
  // the transposed boundary treatment writes the faces' raw cotangent to
  // d_Lb; the reverse pointwise passes read it there and mu elsewhere
  HIPCHK(c, ghk::boundary_vjp(c->d_sh, c->n_shells, c->max_S, c->d_bctab, c->d_gamma, c->d_W, mu, c->d_Lb,
                              c->d_bcg, c->stream));
  {
    Timed t(c, 6);
    HIPCHK(c, ghk::pointwise_vjp(c->d_sh, c->d_blk, c->n_blk, c->d_angtab, c->d_radtab, x, dR, dA, c->d_H,
                                 c->d_dH, c->d_gamma, mu, c->d_Lb, out, c->d_dRb, c->d_dAb, c->d_gpart, c->d_vacc,
                                 (long long)c->P, c->stream));
  }
  {
    Timed t(c, 7);
    HIPCHK(c, launch_plan(c->derivT, c->d_dAb, out,
                        c->stream, 2));
  }
  if (c->maxr)
    HIPCHK(c, ghk::radial_col(c->maxr, c->d_sh, c->d_cblk, c->n_cblk, c->d_dtab, c->d_dRb, out, 0, 50, true, true,
                              c->stream));
  else
    HIPCHK(c, ghk::radial(c->d_sh, c->d_blk, c->n_blk, c->d_dtab, c->d_dRb, out, 0, 50, true, true, c->stream));
  if (g)
    HIPCHK(c, ghk::gamma_reduce(c->d_inst_range, c->d_shell_range, c->n_inst, c->max_S, c->d_gpart, c->d_bcg,
                                c->d_dt, coef, use_dt, g, c->stream));
  return GH_OK;
}

}  // namespace

extern "C" {

int gh_create(gh_ctx** out, int device, void* hip_stream) {
  if (!out) return GH_ERR_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return GH_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return GH_ERR_DEVICE;
  if (lookup_scratch(device) != GH_OK) return GH_ERR_DEVICE;
  gh_ctx* c = new gh_ctx();
  c->device = device;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
    c->n_cu = ncu;
  c->stream = static_cast<hipStream_t>(hip_stream);
  *out = c;
  return GH_OK;
}

int gh_destroy(gh_ctx* c) {
  if (!c) return GH_ERR_ARG;
  free_domain(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  delete c;
  return GH_OK;
}

int gh_set_stream(gh_ctx* c, void* hip_stream) {
  if (!c) return GH_ERR_ARG;
  c->stream = static_cast<hipStream_t>(hip_stream);
  return GH_OK;
}

const char* gh_last_error(const gh_ctx* c) { return c ? c->err.c_str() : "null context"; }

namespace {

// Tensor-coupled filter of the domain (filter_kind 2, 3): per L the analysis /
// synthesis operands and the coupling matrix (and its transpose) cut into
// segments; per L group the columns (shell, radius) of the coefficient array;
// the work list of the coupling kernel; the GEMM groups of PhysToSpec and
// SpecToPhys (maximal runs of consecutive shells with one L).
int build_tensor_filter(gh_ctx* c) {
  int rc;
  const int tens[3][2] = {{0, 10}, {10, 10}, {20, 30}};
  std::vector<TfSeg> segs;
  std::vector<TfCol> colv;
  std::vector<long long> soff[2];
  std::vector<int> swid[2], perm[2], lidx[2];
  std::vector<double> val[2];
  struct Work {
    int seg, col_begin, ncols, nc;
    std::vector<double> slice_cost;
  };
  std::vector<Work> work;
  std::map<int, bool> done;
  // coefficient array offsets per shell
  auto nsp_of = [](int L) { return ((L + 1) * (L + 1) + 1) & ~1; };
  std::vector<long long> xoff(c->n_shells + 1, 0);
  for (int k = 0; k < c->n_shells; ++k) xoff[k + 1] = xoff[k] + 50LL * c->shells[k].n_r * nsp_of(c->shells[k].L);
  if ((rc = dalloc(c, &c->d_tfx, size_t(xoff[c->n_shells])))) return rc;
  if ((rc = dalloc(c, &c->d_tfy, size_t(xoff[c->n_shells])))) return rc;
  {
    // transform form: Legendre tables per L, blocks over (row, s) and (row, i, m'), shell offsets
    std::map<int, long long> lg_off;
    std::vector<double> legtab;
    std::vector<PtBlock> ab, sb;
    for (int k = 0; k < c->n_shells; ++k) {
      const int L = c->shells[k].L, n = L + 1, rows = 50 * c->shells[k].n_r;
      if (!lg_off.count(L)) {
        lg_off[L] = (long long)legtab.size();
        const std::vector<double> T = ghtf::legendre_tables(L);
        legtab.insert(legtab.end(), T.begin(), T.end());
      }
      c->h_sh[k].tf_off = xoff[k];
      c->h_sh[k].lg_off = lg_off[L];
      c->h_sh[k].nsp = nsp_of(L);
      // one thread per (group of 10 rows, coefficient) and (group of 10 rows, m', i)
      for (int q0 = 0; q0 < rows / 10 * n * n; q0 += 256) ab.push_back(PtBlock{k, q0});
      for (int q0 = 0; q0 < rows / 10 * 2 * n * n; q0 += 256) sb.push_back(PtBlock{k, q0});
    }
    if ((rc = upload(c, &c->d_legtab, legtab))) return rc;
    if ((rc = upload(c, &c->d_lg_ablk, ab))) return rc;
    if ((rc = upload(c, &c->d_lg_sblk, sb))) return rc;
    c->n_lg_ablk = int(ab.size());
    c->n_lg_sblk = int(sb.size());
    HIPCHK(c, hipMemcpy(c->d_sh, c->h_sh.data(), c->h_sh.size() * sizeof(ShellDev), hipMemcpyHostToDevice));
  }
  for (int k0 = 0; k0 < c->n_shells; ++k0) {
    const int L = c->shells[k0].L;
    if (done.count(L)) continue;
    done[L] = true;
    const int ns = (L + 1) * (L + 1), S = 2 * ns, nsp = nsp_of(L);
    // B operands: PhysToSpec X = u Ana^T, SpecToPhys u = Y Syn^T; transposes: X = u Syn, u = Y Ana
    const std::vector<double> ana = ghtf::sphere_analysis(L), syn = ghtf::sphere_synthesis(L);
    std::vector<double> anaT(size_t(S) * nsp, 0.0), synT(size_t(ns) * S), synP(size_t(S) * nsp, 0.0);
    for (int s = 0; s < ns; ++s)
      for (int a = 0; a < S; ++a) {
        anaT[size_t(a) * nsp + s] = ana[size_t(s) * S + a];
        synT[size_t(s) * S + a] = syn[size_t(a) * ns + s];
        synP[size_t(a) * nsp + s] = syn[size_t(a) * ns + s];
      }
    double* d = nullptr;
    if ((rc = upload(c, &d, anaT))) return rc;
    c->d_anaT[L] = d;
    if ((rc = upload(c, &d, synT))) return rc;
    c->d_synT[L] = d;
    if ((rc = upload(c, &d, synP))) return rc;
    c->d_syn[L] = d;
    if ((rc = upload(c, &d, ana))) return rc;
    c->d_ana[L] = d;
    const ghtf::Csr F = ghtf::coupling_matrix(L, c->filter_kind, c->filt, false);
    const ghtf::Csr FT = ghtf::transpose(F);
    c->tf_nnz += F.row_ptr.back();
    // columns of this L: every (shell with this L, radius)
    const int col_begin = int(colv.size());
    for (int k = 0; k < c->n_shells; ++k)
      if (c->shells[k].L == L)
        for (int r = 0; r < c->shells[k].n_r; ++r)
          colv.push_back(TfCol{xoff[k] + (long long)r * nsp, (long long)c->shells[k].n_r * nsp});
    const int ncols = int(colv.size()) - col_begin;
    // segments: per tensor, consecutive degrees while the rows fit the
    // 8-column items (a single degree may be larger: fewer columns per item)
    for (auto& tz : tens) {
      const int e0 = tz[0], ne = tz[1];
      for (int l0 = 0; l0 <= L;) {
        int l1 = l0 + 1;
        while (l1 <= L && ne * ((l1 + 1) * (l1 + 1) - l0 * l0) <= 1024) ++l1;
        const int s0 = l0 * l0, nsg = l1 * l1 - s0, n = ne * nsg;
        if (n > TF_MAX_ROWS) return fail(c, GH_ERR_ARG, "tensor filter: L too large for the coupling kernel");
        const int seg_id = int(segs.size()), nslice = (n + 63) / 64;
        segs.push_back(TfSeg{e0, ne, s0, nsg, int(soff[0].size()), 0});
        std::vector<double> cost(nslice, 0.0);
        for (int pass = 0; pass < 2; ++pass) {
          const ghtf::Csr& M = pass ? FT : F;
          auto row_of = [&](int i) { return (long long)(e0 + i / nsg) * ns + s0 + i % nsg; };
          // rows sorted by their number of couplings (longest first)
          std::vector<int> order(n);
          for (int i = 0; i < n; ++i) order[i] = i;
          std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return M.row_ptr[row_of(a) + 1] - M.row_ptr[row_of(a)] > M.row_ptr[row_of(b) + 1] - M.row_ptr[row_of(b)];
          });
          for (int q = 0; q < nslice; ++q) {
            int w = 0;
            for (int lane = 0; lane < 64 && 64 * q + lane < n; ++lane) {
              const long long row = row_of(order[64 * q + lane]);
              w = std::max<int>(w, int(M.row_ptr[row + 1] - M.row_ptr[row]));
            }
            const long long off = (long long)val[pass].size();
            soff[pass].push_back(off);
            swid[pass].push_back(w);
            cost[q] = std::max(cost[q], double(w));
            val[pass].resize(size_t(off) + size_t(64) * w, 0.0);
            lidx[pass].resize(size_t(off) + size_t(64) * w, 0);
            for (int lane = 0; lane < 64; ++lane) {
              const int pos = 64 * q + lane;
              if (pos >= n) {
                perm[pass].push_back(-1);
                continue;
              }
              const int i = order[pos];
              perm[pass].push_back(i);
              const long long row = row_of(i);
              int k = 0;
              for (long long p = M.row_ptr[row]; p < M.row_ptr[row + 1]; ++p, ++k) {
                const int e2 = M.col[p] / ns, s2 = M.col[p] % ns;
                if (e2 < e0 || e2 >= e0 + ne || s2 < s0 || s2 >= s0 + nsg)
                  return fail(c, GH_ERR_DEVICE, "tensor filter: a coupling leaves its segment");
                val[pass][size_t(off) + size_t(64) * k + lane] = M.val[p];
                lidx[pass][size_t(off) + size_t(64) * k + lane] = (e2 - e0) * nsg + (s2 - s0);
              }
            }
          }
        }
        work.push_back(Work{seg_id, col_begin, ncols, tf_cols_for_rows(n), cost});
        l0 = l1;
      }
    }
  }
  // work items per column class: (segment, nc columns, all its slices); the
  // items of one segment go to one XCD (its part of the matrix stays in that
  // XCD's L2), segments balanced over the 8 XCDs; list position p of a launch
  // runs on XCD p % 8.
  std::vector<TfItem> items;
  const int cls_nc[3] = {8, 4, 2};
  for (int cls = 0; cls < 3; ++cls) {
    std::vector<const Work*> ws;
    for (auto& w : work)
      if (w.nc == cls_nc[cls]) ws.push_back(&w);
    std::vector<std::vector<TfItem>> px(8);
    std::vector<std::pair<double, int>> order;
    for (size_t q = 0; q < ws.size(); ++q) {
      double tot = 0.0;
      for (double x : ws[q]->slice_cost) tot += x;
      order.push_back({tot * ws[q]->ncols, int(q)});
    }
    std::sort(order.begin(), order.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
      return a.first > b.first;
    });
    double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (auto& o : order) {
      const Work& w = *ws[o.second];
      const int x = int(std::min_element(load, load + 8) - load);
      load[x] += o.first;
      const int nsl = int(w.slice_cost.size());
      for (int c0 = 0; c0 < w.ncols; c0 += w.nc)
        px[x].push_back(TfItem{w.seg, w.col_begin + c0, std::min(w.nc, w.ncols - c0), 0, nsl, 0, 0, 0});
    }
    size_t longest = 0;
    for (auto& v : px) longest = std::max(longest, v.size());
    const size_t before = items.size();
    for (size_t q = 0; q < longest; ++q)
      for (int x = 0; x < 8; ++x)
        if (q < px[x].size()) items.push_back(px[x][q]);
    c->n_tf_items[cls] = int(items.size() - before);
  }
  if ((rc = upload(c, &c->d_tf_segs, segs))) return rc;
  if ((rc = upload(c, &c->d_tf_cols, colv))) return rc;
  if ((rc = upload(c, &c->d_tf_items, items))) return rc;
  if ((rc = upload(c, &c->d_tf_soff, soff[0]))) return rc;
  if ((rc = upload(c, &c->d_tf_swid, swid[0]))) return rc;
  if ((rc = upload(c, &c->d_tf_perm, perm[0]))) return rc;
  if ((rc = upload(c, &c->d_tfT_perm, perm[1]))) return rc;
  if ((rc = upload(c, &c->d_tf_lidx, lidx[0]))) return rc;
  if ((rc = upload(c, &c->d_tf_val, val[0]))) return rc;
  if ((rc = upload(c, &c->d_tfT_soff, soff[1]))) return rc;
  if ((rc = upload(c, &c->d_tfT_swid, swid[1]))) return rc;
  if ((rc = upload(c, &c->d_tfT_lidx, lidx[1]))) return rc;
  if ((rc = upload(c, &c->d_tfT_val, val[1]))) return rc;
  // GEMM groups
  for (int k = 0; k < c->n_shells;) {
    const int L = c->shells[k].L, ns = (L + 1) * (L + 1), S = 2 * ns, nsp = nsp_of(L);
    int k1 = k, rows = 0;
    while (k1 < c->n_shells && c->shells[k1].L == L) { rows += 50 * c->shells[k1].n_r; ++k1; }
    GemmGroup g;
    g.a_off = 50LL * c->offs[k];
    g.c_off = xoff[k];
    g.B = c->d_anaT[L];
    g.M = rows; g.N = ns; g.K = S;
    g.lda = S; g.ldb = nsp; g.ldc = nsp;
    c->tf_p2s.groups.push_back(g);
    g.B = c->d_syn[L];
    c->tf_p2sT.groups.push_back(g);
    GemmGroup h;
    h.a_off = xoff[k];
    h.c_off = 50LL * c->offs[k];
    h.B = c->d_synT[L];
    h.M = rows; h.N = S; h.K = ns;
    h.lda = nsp; h.ldb = S; h.ldc = S;
    c->tf_s2p.groups.push_back(h);
    h.B = c->d_ana[L];
    c->tf_s2pT.groups.push_back(h);
    k = k1;
  }
  return GH_OK;
}

}  // namespace

int gh_set_domain(gh_ctx* c, int n_inst, int n_shells, const gh_shell* shells, int filter_kind,
                  const double* filter_params) {
  if (!c) return GH_ERR_ARG;
  std::string why;
  int rc = validate_shells(n_inst, n_shells, shells, why);
  if (rc) return fail(c, rc, why);
  if (filter_kind < 0 || filter_kind > 3) return fail(c, GH_ERR_ARG, "filter_kind must be 0, 1, 2 or 3");
  if (filter_kind != 0 && !filter_params) return fail(c, GH_ERR_ARG, "filter_params required for filter_kind 1-3");
  if (filter_kind == 1 || filter_kind == 2) {
    if (!(filter_params[0] >= 0.0 && filter_params[0] < 1.0) || !(filter_params[1] >= 0.0) ||
        !(filter_params[2] > 0.0))
      return fail(c, GH_ERR_ARG, "filter_params: need 0 <= eta_c < 1, alpha >= 0, order > 0");
  }
  if (filter_kind == 3 && !(filter_params[0] >= 0.0))
    return fail(c, GH_ERR_ARG, "filter_params: need eta_c >= 0 for the Heaviside filter");
  HIPCHK(c, hipSetDevice(c->device));
  free_domain(c);
  c->n_inst = n_inst;
  c->n_shells = n_shells;
  c->shells.assign(shells, shells + n_shells);
  c->filter_kind = filter_kind;
  if (filter_kind == 1 || filter_kind == 2) std::memcpy(c->filt, filter_params, 3 * sizeof(double));
  if (filter_kind == 3) c->filt[0] = filter_params[0];

  // layout
  c->offs.assign(n_shells + 1, 0);
  c->max_S = 0;
  for (int k = 0; k < n_shells; ++k) {
    long long S = 2LL * (shells[k].L + 1) * (shells[k].L + 1);
    c->offs[k + 1] = c->offs[k] + shells[k].n_r * S;
    c->max_S = std::max<int>(c->max_S, int(S));
  }
  c->P = c->offs[n_shells];

  // operator caches and tables: radial per n_r, angular per L
  std::map<int, int> d_off, ang_off;
  std::vector<double> dtab, angtab, radtab;
  for (int k = 0; k < n_shells; ++k) {
    int n = shells[k].n_r, L = shells[k].L;
    if (!d_off.count(n)) {
      d_off[n] = int(dtab.size());
      auto D = ghsetup::cgl_diff_matrix(n);
      dtab.insert(dtab.end(), D.begin(), D.end());
    }
    if (!ang_off.count(L)) {
      ang_off[L] = int(angtab.size() / 5);
      auto t = ghsetup::angular_table(L);
      angtab.insert(angtab.end(), t.begin(), t.end());
    }
  }
  std::vector<double> wsum(n_inst, 0.0);
  c->h_sh.assign(n_shells, ShellDev());
  int bc_total = 0;
  for (int k = 0; k < n_shells; ++k) {
    const gh_shell& s = shells[k];
    ShellDev& d = c->h_sh[k];
    d.pt_off = c->offs[k];
    d.n_r = s.n_r;
    d.L = s.L;
    d.n_ph = 2 * (s.L + 1);
    d.S = (s.L + 1) * d.n_ph;
    d.instance = s.instance;
    d.d_off = d_off[s.n_r];
    d.ang_off = ang_off[s.L];
    d.rad_off = int(radtab.size() / 2);
    d.dscale = 2.0 / (s.r_out - s.r_in);
    d.kt_off = -1;
    bool last = (k == n_shells - 1) || shells[k + 1].instance != s.instance;
    bool first = (k == 0) || shells[k - 1].instance != s.instance;
    d.outer = last ? 1 : 0;
    d.inner = first ? 1 : 0;
    d.bc_off = last ? -1 : bc_total;
    if (!last) bc_total += 9 * d.S;
    auto xi = ghsetup::cgl_nodes(s.n_r);
    auto cc = ghsetup::clenshaw_curtis(s.n_r);
    double wang = 0.0;
    {
      std::vector<double> x, w;
      ghsetup::gauss_legendre(s.L, x, w);
      for (double wi : w) wang += wi * 2.0 * 3.14159265358979323846;   // sum over theta, phi
    }
    for (int j = 0; j < s.n_r; ++j) {
      double r = 0.5 * (s.r_in + s.r_out) + 0.5 * (s.r_out - s.r_in) * xi[j];
      double wr = cc[j] * 0.5 * (s.r_out - s.r_in) * r * r;
      radtab.push_back(r);
      radtab.push_back(wr);
      wsum[s.instance] += wr * wang;
    }
  }
  // point blocks (256 points, never straddling shells) and per-instance block ranges
  c->h_blk.clear();
  std::vector<int> range(2 * n_inst, 0);
  for (int k = 0; k < n_shells; ++k) {
    int Pk = int(c->offs[k + 1] - c->offs[k]);
    if (k == 0 || shells[k].instance != shells[k - 1].instance) range[2 * shells[k].instance] = int(c->h_blk.size());
    for (int q0 = 0; q0 < Pk; q0 += 256) c->h_blk.push_back(PtBlock{k, q0});
    range[2 * shells[k].instance + 1] = int(c->h_blk.size());
  }
  c->n_blk = int(c->h_blk.size());
  std::vector<PtBlock> cblk;
  int max_nr = 0;
  for (int k = 0; k < n_shells; ++k) {
    int S = c->h_sh[k].S;
    max_nr = std::max(max_nr, shells[k].n_r);
    for (int a0 = 0; a0 < S; a0 += 256) cblk.push_back(PtBlock{k, a0});
  }
  c->n_cblk = int(cblk.size());
  c->maxr = ghk::radial_col_maxr(max_nr);
  std::vector<PtBlock> fblk;
  for (int k = 0; k + 1 < n_shells; ++k) {
    if (shells[k + 1].instance != shells[k].instance) continue;
    int S = c->h_sh[k].S;
    for (int a0 = 0; a0 < S; a0 += 256) {
      fblk.push_back(PtBlock{k, (shells[k].n_r - 1) * S + a0});
      fblk.push_back(PtBlock{k + 1, a0});
    }
  }
  c->n_fblk = int(fblk.size());

  if ((rc = upload(c, &c->d_sh, c->h_sh))) return rc;
  if ((rc = upload(c, &c->d_blk, c->h_blk))) return rc;
  if ((rc = upload(c, &c->d_cblk, cblk))) return rc;
  if ((rc = upload(c, &c->d_fblk, fblk))) return rc;
  if ((rc = upload(c, &c->d_dtab, dtab))) return rc;
  if ((rc = upload(c, &c->d_angtab, angtab))) return rc;
  if ((rc = upload(c, &c->d_radtab, radtab))) return rc;
  if ((rc = upload(c, &c->d_inst_range, range))) return rc;
  std::vector<int> srange(2 * n_inst, 0);
  for (int k = 0; k < n_shells; ++k) {
    int i = shells[k].instance;
    if (k == 0 || shells[k - 1].instance != i) srange[2 * i] = k;
    srange[2 * i + 1] = k + 1;
  }
  if ((rc = upload(c, &c->d_shell_range, srange))) return rc;
  if ((rc = upload(c, &c->d_wsum, wsum))) return rc;
  if ((rc = dalloc(c, &c->d_bctab, size_t(std::max(bc_total, 1))))) return rc;
  c->bc_total = bc_total;
  if ((rc = dalloc(c, &c->d_partial, size_t(c->n_blk)))) return rc;

  // angular operators (and filters), uploaded once per L
  for (auto& kv : ang_off) {
    int L = kv.first, S = 2 * (L + 1) * (L + 1);
    std::vector<double> none;
    // B operand (Theta^T | Phi^T) of the derivative GEMM, written transposed in place
    std::vector<double> Bop(size_t(S) * 2 * S);
    ghsetup::sphere_operator_into(L, 0, none, true, Bop.data(), size_t(2) * S);
    ghsetup::sphere_operator_into(L, 1, none, true, Bop.data() + S, size_t(2) * S);
    double* d = nullptr;
    if ((rc = upload(c, &d, Bop))) return rc;
    c->d_angop[L] = d;
    // (Theta ; Phi), the B operand of the transposed derivative
    std::vector<double>& BopT = Bop;
    ghsetup::sphere_operator_into(L, 0, none, false, BopT.data(), size_t(S));
    ghsetup::sphere_operator_into(L, 1, none, false, BopT.data() + size_t(S) * S, size_t(S));
    double* dT = nullptr;
    if ((rc = upload(c, &dT, BopT))) return rc;
    c->d_angopT[L] = dT;
    if (filter_kind == 1) {
      auto sig = ghsetup::exp_filter_sigma(L, c->filt[0], c->filt[1], c->filt[2]);
      std::vector<double> F(size_t(S) * S);
      ghsetup::sphere_operator_into(L, 2, sig, true, F.data(), size_t(S));
      double* f = nullptr;
      if ((rc = upload(c, &f, F))) return rc;
      c->d_filtop[L] = f;
      ghsetup::sphere_operator_into(L, 2, sig, false, F.data(), size_t(S));
      double* fT = nullptr;
      if ((rc = upload(c, &fT, F))) return rc;
      c->d_filtopT[L] = fT;
    }
  }

  // GEMM groups: maximal runs of consecutive shells with the same L
  c->deriv.groups.clear();
  c->filter.groups.clear();
  for (int k = 0; k < n_shells;) {
    int L = shells[k].L, S = 2 * (L + 1) * (L + 1);
    int k1 = k, rows = 0;
    while (k1 < n_shells && shells[k1].L == L) { rows += 50 * shells[k1].n_r; ++k1; }
    GemmGroup gd;
    gd.a_off = 50LL * c->offs[k];
    gd.c_off = 100LL * c->offs[k];
    gd.B = c->d_angop[L];
    gd.M = rows; gd.N = 2 * S; gd.K = S;
    gd.lda = S; gd.ldb = 2 * S; gd.ldc = 2 * S;
    c->deriv.groups.push_back(gd);
    GemmGroup gt;                      // transposed derivative: [50 n_r x 2S] (Theta ; Phi) -> [50 n_r x S]
    gt.a_off = 100LL * c->offs[k];
    gt.c_off = 50LL * c->offs[k];
    gt.B = c->d_angopT[L];
    gt.M = rows; gt.N = S; gt.K = 2 * S;
    gt.lda = 2 * S; gt.ldb = S; gt.ldc = S;
    c->derivT.groups.push_back(gt);
    if (filter_kind == 1) {
      GemmGroup gf = gd;
      gf.c_off = 50LL * c->offs[k];
      gf.B = c->d_filtop[L];
      gf.N = S; gf.ldb = S; gf.ldc = S;
      c->filter.groups.push_back(gf);
      GemmGroup gft = gf;
      gft.B = c->d_filtopT[L];
      c->filterT.groups.push_back(gft);
    }
    k = k1;
  }

  if (filter_kind >= 2 && (rc = build_tensor_filter(c))) return rc;

  // work space
  size_t F50 = size_t(50) * c->P;
  if ((rc = dalloc(c, &c->d_dR, F50))) return rc;
  if ((rc = dalloc(c, &c->d_dA, 2 * F50))) return rc;
  if ((rc = dalloc(c, &c->d_W, F50))) return rc;
  if ((rc = dalloc(c, &c->d_ua, F50))) return rc;
  if ((rc = dalloc(c, &c->d_ub, F50))) return rc;
  if ((rc = dalloc(c, &c->d_H, size_t(4) * c->P))) return rc;
  if ((rc = dalloc(c, &c->d_dH, size_t(16) * c->P))) return rc;
  if ((rc = dalloc(c, &c->d_gamma, size_t(3) * n_inst))) return rc;
  if ((rc = dalloc(c, &c->d_dt, size_t(n_inst)))) return rc;
  // tile shapes: pick the fastest for this domain, timed on non-zero data
  HIPCHK(c, ghk::fill_pattern(c->d_ua, (long long)F50, c->stream));
  if ((rc = autotune(c, c->deriv, c->d_ua, c->d_dA, 0))) return rc;
  if (filter_kind == 1)
    if ((rc = autotune(c, c->filter, c->d_ua, c->d_ub, 1))) return rc;
  if (filter_kind >= 2) {
    if ((rc = autotune(c, c->tf_p2s, c->d_ua, c->d_tfx, 6))) return rc;
    if ((rc = autotune(c, c->tf_s2p, c->d_tfx, c->d_ub, 7))) return rc;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->have_domain = true;
  return GH_OK;
}

int gh_num_points(const gh_ctx* c, long long* total, long long* offsets) {
  if (!c || !total) return GH_ERR_ARG;
  if (!c->have_domain) return GH_ERR_ORDER;
  *total = c->P;
  if (offsets)
    for (int k = 0; k <= c->n_shells; ++k) offsets[k] = c->offs[k];
  return GH_OK;
}

int gh_set_background(gh_ctx* c, const double* H, const double* dH, const double* u_bg) {
  if (!c) return GH_ERR_ARG;
  if (!c->have_domain) return fail(c, GH_ERR_ORDER, "gh_set_domain has not been called");
  if (!H || !dH || !u_bg) return fail(c, GH_ERR_ARG, "H, dH and u_bg must be device pointers");
  HIPCHK(c, hipSetDevice(c->device));
  c->have_bg = false;
  // scratch for the checks lives in the work space (d_partial holds >= 1 double,
  // d_W >= 50 P doubles); nothing is queued on them concurrently in setup
  int* d_cnt = reinterpret_cast<int*>(c->d_partial);
  HIPCHK(c, hipMemsetAsync(d_cnt, 0, sizeof(int), c->stream));
  HIPCHK(c, ghk::nonfinite_count(H, 4 * c->P, d_cnt, c->stream));
  HIPCHK(c, ghk::nonfinite_count(dH, 16 * c->P, d_cnt, c->stream));
  HIPCHK(c, ghk::nonfinite_count(u_bg, 50 * c->P, d_cnt, c->stream));
  int cnt = 0;
  HIPCHK(c, hipMemcpyAsync(&cnt, d_cnt, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (cnt) return fail(c, GH_ERR_NONFINITE, std::to_string(cnt) + " non-finite background values");
  HIPCHK(c, hipMemcpyAsync(c->d_H, H, 4 * c->P * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_dH, dH, 16 * c->P * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  size_t nex = size_t(c->n_shells) * c->max_S;
  if (nex > size_t(50) * c->P) return fail(c, GH_ERR_ARG, "internal: excision scratch too small");
  double* d_ex = c->d_W;
  HIPCHK(c, ghk::bc_setup(c->d_sh, c->n_shells, c->max_S, c->d_angtab, u_bg, c->d_bctab, d_ex, c->stream));
  std::vector<double> ex(nex);
  HIPCHK(c, hipMemcpyAsync(ex.data(), d_ex, nex * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double mn = INFINITY;
  for (double v : ex) mn = std::min(mn, v);
  if (!(mn >= 0.0)) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "excision boundary is not pure outflow (min characteristic speed %.6g)", mn);
    return fail(c, GH_ERR_NOT_OUTFLOW, buf);
  }
  c->have_bg = true;
  return GH_OK;
}

int gh_set_params(gh_ctx* c, const double* gamma, const double* dt) {
  if (!c) return GH_ERR_ARG;
  if (!c->have_domain) return fail(c, GH_ERR_ORDER, "gh_set_domain has not been called");
  if (!gamma) return fail(c, GH_ERR_ARG, "gamma must be a host pointer [n_inst][3]");
  for (int i = 0; i < 3 * c->n_inst; ++i)
    if (!std::isfinite(gamma[i])) return fail(c, GH_ERR_NONFINITE, "non-finite gamma");
  if (dt)
    for (int i = 0; i < c->n_inst; ++i)
      if (!std::isfinite(dt[i]) || !(dt[i] > 0.0)) return fail(c, GH_ERR_ARG, "dt must be finite and > 0");
  HIPCHK(c, hipSetDevice(c->device));
  // Work already queued (on the context's stream, or graph replays on the
  // capture stream) reads gamma and dt from device memory: let it finish
  // before they change.  A plain hipMemcpy would only be ordered against the
  // null stream, not against a non-blocking caller stream.
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->cap_stream) HIPCHK(c, hipStreamSynchronize(c->cap_stream));
  HIPCHK(c, hipMemcpy(c->d_gamma, gamma, 3 * c->n_inst * sizeof(double), hipMemcpyHostToDevice));
  c->have_gamma = true;
  if (dt) {
    HIPCHK(c, hipMemcpy(c->d_dt, dt, c->n_inst * sizeof(double), hipMemcpyHostToDevice));
    c->have_dt = true;
  }
  return GH_OK;
}

int gh_rhs(gh_ctx* c, const double* u, double* dudt) {
  int rc = check_ready(c, false);
  if (rc) return rc;
  if (!u || !dudt || u == dudt) return fail(c, GH_ERR_ARG, "u and dudt must be distinct device pointers");
  HIPCHK(c, hipSetDevice(c->device));
  return queue_rhs(c, u, dudt);
}

int gh_step(gh_ctx* c, double* u, int n_steps) {
  int rc = check_ready(c, true);
  if (rc) return rc;
  if (!u || n_steps < 0) return fail(c, GH_ERR_ARG, "need u != NULL and n_steps >= 0");
  HIPCHK(c, hipSetDevice(c->device));
  if (n_steps == 0) return GH_OK;
  if (!c->use_graph || c->timing) {
    for (int n = 0; n < n_steps; ++n)
      if ((rc = queue_step(c, u))) return rc;
    return GH_OK;
  }
  // graph path: capture one step on the library's own stream (the caller's
  // stream may be the legacy default stream, which cannot be captured), then
  // replay it n_steps times, ordered after / before the caller's work by events
  if (c->graph_u != u) {
    drop_graph(c);
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    rc = queue_step(c, u);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->stream = user;
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(c, GH_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    c->graph = g;
    HIPCHK(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
    c->graph_u = u;
  }
  HIPCHK(c, hipEventRecord(c->ev_in, c->stream));
  HIPCHK(c, hipStreamWaitEvent(c->cap_stream, c->ev_in, 0));
  for (int n = 0; n < n_steps; ++n) HIPCHK(c, hipGraphLaunch(c->graph_exec, c->cap_stream));
  HIPCHK(c, hipEventRecord(c->ev_out, c->cap_stream));
  HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_out, 0));
  return GH_OK;
}

namespace {

// Tables, work space and tuned GEMM plans of the transform path.
int ensure_transform(gh_ctx* c) {
  if (c->have_tr) return GH_OK;
  int rc;
  std::map<int, long long> kt_off;
  std::vector<double> ktab;
  for (int k = 0; k < c->n_shells; ++k) {
    const int L = c->shells[k].L;
    if (kt_off.count(L)) continue;
    kt_off[L] = (long long)ktab.size();
    std::vector<double> none;
    for (int which = 0; which < 3; ++which) {
      std::vector<double> sig = (which == 2 && c->filter_kind == 1)
                                    ? ghsetup::exp_filter_sigma(L, c->filt[0], c->filt[1], c->filt[2])
                                    : std::vector<double>(L + 1, 1.0);
      auto K = ghsetup::sphere_factors(L, which, sig);
      ktab.insert(ktab.end(), K.begin(), K.end());
    }
    const int n = L + 1;
    auto T = ghsetup::fourier_table(L);
    std::vector<double> TT(T.size());
    for (int a = 0; a < 2 * n; ++a)
      for (int b = 0; b < 2 * n; ++b) TT[size_t(b) * 2 * n + a] = T[size_t(a) * 2 * n + b];
    double *dA = nullptr, *dS = nullptr;
    if ((rc = upload(c, &dA, T))) return rc;
    if ((rc = upload(c, &dS, TT))) return rc;
    c->d_fana[L] = dA;
    c->d_fsyn[L] = dS;
  }
  if ((rc = upload(c, &c->d_ktab, ktab))) return rc;
  // per order transposed ([kind][m][i'][i]) for the matrix-core theta step
  std::vector<double> ktabT(ktab.size());
  for (const auto& kv : kt_off) {
    const int n = kv.first + 1;
    const long long n2 = (long long)n * n;
    for (long long km = 0; km < 3LL * n; ++km)
      for (int i = 0; i < n; ++i)
        for (int ip = 0; ip < n; ++ip) ktabT[kv.second + km * n2 + (long long)ip * n + i] = ktab[kv.second + km * n2 + (long long)i * n + ip];
  }
  if ((rc = upload(c, &c->d_ktabT, ktabT))) return rc;
  for (int k = 0; k < c->n_shells; ++k) c->h_sh[k].kt_off = kt_off[c->shells[k].L];
  HIPCHK(c, hipMemcpy(c->d_sh, c->h_sh.data(), c->h_sh.size() * sizeof(ShellDev), hipMemcpyHostToDevice));
  if ((rc = dalloc(c, &c->d_X, size_t(100) * c->P))) return rc;
  // theta step: shells with n = L + 1 a multiple of 16 on the matrix cores
  // (items of 8 rows x 8 or 16 orders, per n); the others in blocks of 16 (field,
  // radius) rows x 256 (node, column) pairs
  std::vector<PtBlock> tb;
  std::vector<ThetaItem> ti[4];
  int maxn = 0;
  for (int k = 0; k < c->n_shells; ++k) {
    const int S = c->h_sh[k].S, rows = 50 * c->shells[k].n_r, n = c->shells[k].L + 1;
    if (n % 16 == 0) {
      // Workgroups go round-robin over the 8 XCDs, so the items are ordered
      // in groups of 8 row blocks, order block after order block: every
      // order block of a row block then runs on the same XCD in consecutive
      // rounds.  With 8-order items the half 128-byte lines each one writes
      // (and reads) meet in that XCD's L2; 16-order items move whole lines.
      // Groups are padded to 8 (r0 = -1: no work).
      std::vector<ThetaItem>& v = ti[n / 16 - 1];
      while (v.size() % 8) v.push_back(ThetaItem{k, -1, 0, 0});
      const int nrb = (rows + 7) / 8, mb = ghk::theta_item_orders(n);
      for (int g0 = 0; g0 < nrb; g0 += 8)
        for (int m0 = 0; m0 < n; m0 += mb)
          for (int rb = g0; rb < g0 + 8; ++rb) v.push_back(ThetaItem{k, rb < nrb ? 8 * rb : -1, m0, 0});
      continue;
    }
    maxn = std::max(maxn, n);
    for (int r0 = 0; r0 < rows; r0 += 16)
      for (int a0 = 0; a0 < S; a0 += 256) tb.push_back(PtBlock{k, r0 * S + a0});
  }
  c->tr_nmax = maxn <= 16 ? 16 : (maxn <= 32 ? 32 : 64);
  c->n_tblk = int(tb.size());
  if (!tb.empty() && (rc = upload(c, &c->d_tblk, tb))) return rc;
  for (int g = 0; g < 4; ++g) {
    c->n_titem[g] = int(ti[g].size());
    if (!ti[g].empty() && (rc = upload(c, &c->d_titem[g], ti[g]))) return rc;
  }
  // plans over maximal runs of consecutive shells with the same L: a state is
  // a [rows * n x 2n] matrix (rows = (field, radius) pairs), the theta output a
  // [rows * 2n x 2n] one laid out like the angular derivatives
  for (int k = 0; k < c->n_shells;) {
    const int L = c->shells[k].L, n = L + 1;
    int k1 = k, rows = 0;
    while (k1 < c->n_shells && c->shells[k1].L == L) { rows += 50 * c->shells[k1].n_r; ++k1; }
    GemmGroup ga;
    ga.a_off = 50LL * c->offs[k];
    ga.c_off = 50LL * c->offs[k];
    ga.B = c->d_fana[L];
    ga.M = rows * n; ga.N = 2 * n; ga.K = 2 * n;
    ga.lda = 2 * n; ga.ldb = 2 * n; ga.ldc = 2 * n;
    c->tr_ana.groups.push_back(ga);
    GemmGroup gs = ga;
    gs.a_off = 100LL * c->offs[k];
    gs.c_off = 100LL * c->offs[k];
    gs.B = c->d_fsyn[L];
    gs.M = rows * 2 * n;
    c->tr_syn.groups.push_back(gs);
    GemmGroup gf = ga;
    gf.B = c->d_fsyn[L];
    c->tr_fsyn.groups.push_back(gf);
    k = k1;
  }
  const size_t F50 = size_t(50) * c->P;
  HIPCHK(c, ghk::fill_pattern(c->d_ua, (long long)F50, c->stream));
  HIPCHK(c, ghk::fill_pattern(c->d_X, (long long)(2 * F50), c->stream));
  if ((rc = autotune(c, c->tr_ana, c->d_ua, c->d_ub, 4))) return rc;
  if ((rc = autotune(c, c->tr_syn, c->d_X, c->d_dA, 5))) return rc;
  if (c->filter_kind != 0)
    if ((rc = autotune(c, c->tr_fsyn, c->d_X, c->d_ub, 5))) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->have_tr = true;
  return GH_OK;
}

}  // namespace

namespace {

// Average time of 5 launches of op (after one untimed) on the context's stream.
int time_op(gh_ctx* c, const std::function<int()>& op, float* ms) {
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  int rc = op();
  if (rc) return rc;
  HIPCHK(c, hipEventRecord(e0, c->stream));
  for (int it = 0; it < 5; ++it)
    if ((rc = op())) return rc;
  HIPCHK(c, hipEventRecord(e1, c->stream));
  HIPCHK(c, hipEventSynchronize(e1));
  HIPCHK(c, hipEventElapsedTime(ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return GH_OK;
}

}  // namespace

int gh_set_angular(gh_ctx* c, int method) {
  if (!c) return GH_ERR_ARG;
  if (!c->have_domain) return fail(c, GH_ERR_ORDER, "gh_set_domain has not been called");
  if (method < 0 || method > 2) return fail(c, GH_ERR_ARG, "method must be 0 (dense), 1 (transform) or 2 (faster)");
  HIPCHK(c, hipSetDevice(c->device));
  int rc;
  if (method >= 1 && (rc = ensure_transform(c))) return rc;
  bool dtr = method == 1, ftr = method == 1 && c->filter_kind != 0;
  if (method == 2) {
    // time both forms of each operation on this domain (non-zero data in the work arrays)
    const bool timing = c->timing;
    c->timing = false;
    HIPCHK(c, ghk::fill_pattern(c->d_ua, (long long)(size_t(50) * c->P), c->stream));
    float t_dense = 0, t_tr = 0;
    c->deriv_tr = false;
    if ((rc = time_op(c, [&]() { return queue_derivs(c, c->d_ua); }, &t_dense))) return rc;
    c->deriv_tr = true;
    if ((rc = time_op(c, [&]() { return queue_derivs(c, c->d_ua); }, &t_tr))) return rc;
    dtr = t_tr < t_dense;
    if (c->filter_kind != 0) {
      c->filt_tr = false;
      if ((rc = time_op(c, [&]() { return queue_filter(c, c->d_ua, c->d_ub); }, &t_dense))) return rc;
      c->filt_tr = true;
      if ((rc = time_op(c, [&]() { return queue_filter(c, c->d_ua, c->d_ub); }, &t_tr))) return rc;
      ftr = t_tr < t_dense;
    }
    c->timing = timing;
  }
  if (method != c->ang_method || dtr != c->deriv_tr || ftr != c->filt_tr) drop_graph(c);
  c->ang_method = method;
  c->deriv_tr = dtr;
  c->filt_tr = ftr;
  return GH_OK;
}

int gh_set_graph(gh_ctx* c, int enable) {
  if (!c) return GH_ERR_ARG;
  HIPCHK(c, hipSetDevice(c->device));
  drop_graph(c);
  if (enable && !c->cap_stream) {
    HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
  }
  c->use_graph = enable != 0;
  return GH_OK;
}

int gh_constraints(gh_ctx* c, const double* u, double* C, double* norm) {
  if (!c) return GH_ERR_ARG;
  if (!c->have_domain) return fail(c, GH_ERR_ORDER, "gh_set_domain has not been called");
  if (!c->have_bg) return fail(c, GH_ERR_ORDER, "gh_set_background has not been called");
  if (!u) return fail(c, GH_ERR_ARG, "u must be a device pointer");
  HIPCHK(c, hipSetDevice(c->device));
  int rc = queue_derivs(c, u);
  if (rc) return rc;
  HIPCHK(c, ghk::constraints(c->d_sh, c->d_blk, c->n_blk, c->d_angtab, c->d_radtab, u, c->d_dR, c->d_dA, c->d_H,
                             C, c->d_partial, c->stream));
  if (norm) HIPCHK(c, ghk::reduce_norm(c->d_inst_range, c->n_inst, c->d_partial, c->d_wsum, norm, c->stream));
  return GH_OK;
}

int gh_constraints_static(gh_ctx* c, const double* u, double* C, double* norm) {
  if (!c) return GH_ERR_ARG;
  if (!c->have_domain) return fail(c, GH_ERR_ORDER, "gh_set_domain has not been called");
  if (!c->have_bg) return fail(c, GH_ERR_ORDER, "gh_set_background has not been called");
  if (!u) return fail(c, GH_ERR_ARG, "u must be a device pointer");
  if (c->n_blk > GH_STATIC_SCRATCH_DOUBLES)
    return fail(c, GH_ERR_ARG, "the domain has " + std::to_string(c->n_blk) + " point blocks of 256; the static "
                "scratch holds the partial sums of at most " + std::to_string(GH_STATIC_SCRATCH_DOUBLES));
  double* part = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch_ptr[c->device] : nullptr;
  if (!part) return fail(c, GH_ERR_DEVICE, "no scratch address for this device");
  HIPCHK(c, hipSetDevice(c->device));
  // kernel timing would create events; none are created here
  const bool timing = c->timing;
  c->timing = false;
  int rc = queue_derivs(c, u);
  c->timing = timing;
  if (rc) return rc;
  // every block writes its own partial sum, so nothing needs clearing
  HIPCHK(c, ghk::constraints(c->d_sh, c->d_blk, c->n_blk, c->d_angtab, c->d_radtab, u, c->d_dR, c->d_dA, c->d_H,
                             C, part, c->stream));
  if (norm) HIPCHK(c, ghk::reduce_norm(c->d_inst_range, c->n_inst, part, c->d_wsum, norm, c->stream));
  return GH_OK;
}

int gh_rhs_vjp(gh_ctx* c, const double* u, const double* lam, double* lam_u, double* g_gamma) {
  int rc = check_ready(c, false);
  if (rc) return rc;
  if (!u || !lam || !lam_u || lam_u == u || lam_u == lam)
    return fail(c, GH_ERR_ARG, "u, lam, lam_u must be device pointers and lam_u distinct from u and lam");
  if (c->iface_mode)
    return fail(c, GH_ERR_ARG, "the reverse pass needs the frozen interface projection (gh_set_interface 0)");
  if (c->outer_mode)
    return fail(c, GH_ERR_ARG, "the reverse pass needs the Dirichlet outer boundary (gh_set_outer_bc 0)");
  HIPCHK(c, hipSetDevice(c->device));
  if ((rc = ensure_adjoint(c))) return rc;
  return queue_rhs_vjp(c, u, lam, lam_u, 1.0, 0, g_gamma);
}

// Reverse sweep of one RK3 step given its stage states u1, u2.
int queue_step_vjp(gh_ctx* c, const double* u_n, const double* u1, const double* u2, const double* lam_np1,
                   double* lam_n, double* g_gamma, const double* kept = nullptr) {
  int rc;
  const size_t F150 = size_t(150) * c->P;
  const double* k0 = kept ? kept : nullptr;
  const double* k1 = kept ? kept + F150 : nullptr;
  const double* k2 = kept ? kept + 2 * F150 : nullptr;
  // filter: u_{n+1} = F u3, so lam3 = F^T lam_{n+1}
  const double* lam3 = lam_np1;
  if (c->filter_kind == 1) {
    HIPCHK(c, launch_plan(c->filterT, lam_np1,
                        c->d_lam3, c->stream, 3));
    lam3 = c->d_lam3;
  } else if (c->filter_kind >= 2) {
    if ((rc = queue_tensor_filter(c, lam_np1, c->d_lam3, true))) return rc;
    lam3 = c->d_lam3;
  }
  // u3 = 1/3 u + 2/3 (u2 + h L(u2))
  if ((rc = queue_rhs_vjp(c, u2, lam3, c->d_T, 2.0 / 3.0, 1, g_gamma, k2))) return rc;
  LINCOMB(ghk::lincomb(c->d_sh, c->d_blk, c->n_blk, c->d_dt, 1, 0.0, nullptr, 2.0 / 3.0, lam3, 2.0 / 3.0, c->d_T,
                         c->d_mu2, c->stream));
  // u2 = 3/4 u + 1/4 (u1 + h L(u1))
  if ((rc = queue_rhs_vjp(c, u1, c->d_mu2, c->d_T, 0.25, 1, g_gamma, k1))) return rc;
  LINCOMB(ghk::lincomb(c->d_sh, c->d_blk, c->n_blk, c->d_dt, 1, 0.0, nullptr, 0.25, c->d_mu2, 0.25, c->d_T,
                         c->d_mu1, c->stream));
  // u1 = u + h L(u)
  if ((rc = queue_rhs_vjp(c, u_n, c->d_mu1, c->d_T, 1.0, 1, g_gamma, k0))) return rc;
  LINCOMB(ghk::lincomb(c->d_sh, c->d_blk, c->n_blk, c->d_dt, 0, 1.0 / 3.0, lam3, 0.75, c->d_mu2, 0.0, nullptr,
                         lam_n, c->stream));
  LINCOMB(ghk::lincomb(c->d_sh, c->d_blk, c->n_blk, c->d_dt, 1, 1.0, lam_n, 1.0, c->d_mu1, 1.0, c->d_T, lam_n,
                         c->stream));
  return GH_OK;
}

int gh_step_vjp(gh_ctx* c, const double* u_n, const double* lam_np1, double* lam_n, double* g_gamma) {
  int rc = check_ready(c, true);
  if (rc) return rc;
  if (!u_n || !lam_np1 || !lam_n || lam_n == u_n)
    return fail(c, GH_ERR_ARG, "u_n, lam_np1, lam_n must be device pointers and lam_n distinct from u_n");
  if (c->iface_mode)
    return fail(c, GH_ERR_ARG, "the reverse pass needs the frozen interface projection (gh_set_interface 0)");
  if (c->outer_mode)
    return fail(c, GH_ERR_ARG, "the reverse pass needs the Dirichlet outer boundary (gh_set_outer_bc 0)");
  HIPCHK(c, hipSetDevice(c->device));
  if ((rc = ensure_adjoint(c))) return rc;
  // recompute the stages: u1 = u + h L(u), u2 = 3/4 u + 1/4 (u1 + h L(u1))
  if ((rc = queue_stage(c, 0.0, nullptr, 1.0, u_n, c->d_u1))) return rc;
  if ((rc = queue_stage(c, 0.75, u_n, 0.25, c->d_u1, c->d_u2))) return rc;
  return queue_step_vjp(c, u_n, c->d_u1, c->d_u2, lam_np1, lam_n, g_gamma);
}

int gh_step_stages(gh_ctx* c, double* u, double* u1, double* u2, double* derivs) {
  int rc = check_ready(c, true);
  if (rc) return rc;
  if (!u || !u1 || !u2 || u1 == u || u2 == u || u1 == u2)
    return fail(c, GH_ERR_ARG, "u, u1, u2 must be distinct device pointers");
  if (derivs && (derivs == u || derivs == u1 || derivs == u2))
    return fail(c, GH_ERR_ARG, "derivs must not alias u, u1 or u2");
  HIPCHK(c, hipSetDevice(c->device));
  const bool filt = c->filter_kind != 0;
  const size_t F150 = size_t(150) * c->P;
  if ((rc = queue_stage(c, 0.0, nullptr, 1.0, u, u1, derivs))) return rc;
  if ((rc = queue_stage(c, 0.75, u, 0.25, u1, u2, derivs ? derivs + F150 : nullptr))) return rc;
  double* dst = filt ? c->d_ua : u;
  if ((rc = queue_stage(c, 1.0 / 3.0, u, 2.0 / 3.0, u2, dst, derivs ? derivs + 2 * F150 : nullptr))) return rc;
  if (filt)
    if ((rc = queue_filter(c, c->d_ua, u))) return rc;
  return GH_OK;
}

int gh_step_vjp_stages(gh_ctx* c, const double* u_n, const double* u1, const double* u2, const double* derivs,
                       const double* lam_np1, double* lam_n, double* g_gamma) {
  int rc = check_ready(c, true);
  if (rc) return rc;
  if (!u_n || !u1 || !u2 || !lam_np1 || !lam_n || lam_n == u_n || lam_n == u1 || lam_n == u2 ||
      (derivs && lam_n == derivs))
    return fail(c, GH_ERR_ARG, "device pointers required; lam_n must not alias u_n, u1, u2 or derivs");
  if (c->iface_mode)
    return fail(c, GH_ERR_ARG, "the reverse pass needs the frozen interface projection (gh_set_interface 0)");
  if (c->outer_mode)
    return fail(c, GH_ERR_ARG, "the reverse pass needs the Dirichlet outer boundary (gh_set_outer_bc 0)");
  HIPCHK(c, hipSetDevice(c->device));
  if ((rc = ensure_adjoint(c))) return rc;
  return queue_step_vjp(c, u_n, u1, u2, lam_np1, lam_n, g_gamma, derivs);
}

// Dormand-Prince 5(4) tableau (Dormand & Prince 1980): stage weights a_ij,
// fifth-order weights (row 7) and error weights (fifth minus embedded fourth order).
namespace dp5c {
const double A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
const double E[7] = {35.0 / 384 - 5179.0 / 57600, 0, 500.0 / 1113 - 7571.0 / 16695, 125.0 / 192 - 393.0 / 640,
                     -2187.0 / 6784 + 92097.0 / 339200, 11.0 / 84 - 187.0 / 2100, -1.0 / 40};
}  // namespace dp5c

int ensure_dp5(gh_ctx* c) {
  if (c->have_dp5) return GH_OK;
  const size_t F50 = size_t(50) * c->P;
  int rc;
  if ((rc = dalloc(c, &c->d_dpk, 7 * F50))) return rc;
  if ((rc = dalloc(c, &c->d_dpy, F50))) return rc;
  if ((rc = dalloc(c, &c->d_dpu5, F50))) return rc;
  if (c->filter_kind != 0 && (rc = dalloc(c, &c->d_dpf, F50))) return rc;
  if ((rc = dalloc(c, &c->d_dprej, size_t(c->n_inst)))) return rc;
  if ((rc = dalloc(c, &c->d_dpacc, size_t(c->n_inst)))) return rc;
  std::vector<double> nval(c->n_inst, 0.0);
  for (int k = 0; k < c->n_shells; ++k) nval[c->shells[k].instance] += 50.0 * double(c->offs[k + 1] - c->offs[k]);
  if ((rc = upload(c, &c->d_dpnval, nval))) return rc;
  c->have_dp5 = true;
  return GH_OK;
}

int gh_constraints_vjp(gh_ctx* c, const double* u, const double* lam_norm, double* lam_u) {
  if (!c) return GH_ERR_ARG;
  if (!c->have_domain) return fail(c, GH_ERR_ORDER, "gh_set_domain has not been called");
  if (!c->have_bg) return fail(c, GH_ERR_ORDER, "gh_set_background has not been called");
  if (!u || !lam_norm || !lam_u || lam_u == u)
    return fail(c, GH_ERR_ARG, "u, lam_norm, lam_u must be device pointers and lam_u distinct from u");
  HIPCHK(c, hipSetDevice(c->device));
  int rc = ensure_adjoint(c);
  if (rc) return rc;
  if ((rc = queue_derivs(c, u))) return rc;
  HIPCHK(c, ghk::constraints(c->d_sh, c->d_blk, c->n_blk, c->d_angtab, c->d_radtab, u, c->d_dR, c->d_dA, c->d_H,
                             c->d_C, c->d_partial, c->stream));
  HIPCHK(c, ghk::reduce_norm(c->d_inst_range, c->n_inst, c->d_partial, c->d_wsum, c->d_norm, c->stream));
  HIPCHK(c, ghk::constraints_vjp(c->d_sh, c->d_blk, c->n_blk, c->d_angtab, c->d_radtab, u, c->d_H, c->d_C, c->d_norm,
                                 c->d_wsum, lam_norm, lam_u, c->d_dRb, c->d_dAb, c->stream));
  HIPCHK(c, launch_plan(c->derivT, c->d_dAb, lam_u,
                      c->stream, 2));
  if (c->maxr)
    HIPCHK(c, ghk::radial_col(c->maxr, c->d_sh, c->d_cblk, c->n_cblk, c->d_dtab, c->d_dRb, lam_u, 0, 50, true, true,
                              c->stream));
  else
    HIPCHK(c, ghk::radial(c->d_sh, c->d_blk, c->n_blk, c->d_dtab, c->d_dRb, lam_u, 0, 50, true, true, c->stream));
  return GH_OK;
}

int gh_set_gemm_variant(gh_ctx* c, int plan, int shape, int order) {
  if (!c) return GH_ERR_ARG;
  if (!c->have_domain) return fail(c, GH_ERR_ORDER, "gh_set_domain has not been called");
  if (plan < 0 || plan > 1 || shape < 0 || shape >= ghk::NUM_TILE_SHAPES || order < 0 ||
      order >= ghk::NUM_TILE_ORDERS)
    return fail(c, GH_ERR_ARG, "plan 0 or 1, shape 0 .. NUM_TILE_SHAPES-1, order 0 .. 2");
  if (plan == 1 && c->filter_kind != 1) return fail(c, GH_ERR_ARG, "the domain has no filter GEMM (filter_kind 1)");
  if (!ghk::shape_fits(shape, (plan ? c->filter : c->deriv).groups))
    return fail(c, GH_ERR_ARG, "this variant loads directly into LDS and needs even K, N, lda, ldb and offsets");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  drop_graph(c);
  return plan_upload(c, plan ? c->filter : c->deriv, shape, order);
}

int gh_set_gemm_plan(gh_ctx* c, int plan, int shape, int order, int tail_shape, int tail_chunks, int round) {
  if (!c) return GH_ERR_ARG;
  if (!c->have_domain) return fail(c, GH_ERR_ORDER, "gh_set_domain has not been called");
  if (plan < 0 || plan > 10) return fail(c, GH_ERR_ARG, "plan must be 0 .. 10");
  if (shape < 0 || shape >= ghk::NUM_TILE_SHAPES || order < 0 || order >= ghk::NUM_TILE_ORDERS)
    return fail(c, GH_ERR_ARG, "shape 0 .. NUM_TILE_SHAPES-1, order 0 .. 2");
  if (tail_shape >= ghk::NUM_TILE_SHAPES || (tail_shape >= 0 && (tail_chunks < 1 || tail_chunks > 8)) || round < 0)
    return fail(c, GH_ERR_ARG, "tail_shape -1 (one launch) or 0 .. NUM_TILE_SHAPES-1 with 1 .. 8 K chunks; round >= 0");
  HIPCHK(c, hipSetDevice(c->device));
  int rc;
  if ((plan == 2 || plan == 3 || plan >= 9) && (rc = ensure_adjoint(c))) return rc;
  if (plan >= 4 && plan <= 6 && !c->have_tr)
    return fail(c, GH_ERR_ORDER, "the transform plans exist after gh_set_angular 1 or 2");
  GemmPlan* const plans[11] = {&c->deriv, &c->filter, &c->derivT, &c->filterT, &c->tr_ana, &c->tr_syn,
                               &c->tr_fsyn, &c->tf_p2s, &c->tf_s2p, &c->tf_p2sT, &c->tf_s2pT};
  GemmPlan& pl = *plans[plan];
  if (pl.groups.empty()) return fail(c, GH_ERR_ARG, "this domain has no such GEMM plan");
  if (!ghk::shape_fits(shape, pl.groups))
    return fail(c, GH_ERR_ARG, "this variant loads directly into LDS and needs even K, N, lda, ldb and offsets");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  drop_graph(c);
  if (tail_shape < 0) return plan_upload(c, pl, shape, order);
  std::vector<GemmGroup> mainv, tailv;
  if (!split_rows(pl.groups, shape, round > 0 ? round : c->n_cu, mainv, tailv) || tailv.size() != 1)
    return fail(c, GH_ERR_ARG, "no split of this plan's tiles into whole rounds of that size and one tail group");
  if (tailv[0].K < 16 * tail_chunks) return fail(c, GH_ERR_ARG, "the tail's K is too short for that many chunks");
  if (!ghk::shape_fits(tail_shape, tailv))
    return fail(c, GH_ERR_ARG, "the tail variant loads directly into LDS and needs even K, N, lda, ldb and offsets");
  return plan_upload_split(c, pl, mainv, tailv[0], shape, order, tail_shape, tail_chunks);
}

int gh_set_outer_bc(gh_ctx* c, int mode) {
  if (!c) return GH_ERR_ARG;
  if (!c->have_domain) return fail(c, GH_ERR_ORDER, "gh_set_domain has not been called");
  if (mode != 0 && mode != 1) return fail(c, GH_ERR_ARG, "mode must be 0 (Dirichlet) or 1 (constraint-preserving)");
  if (mode != c->outer_mode) drop_graph(c);
  c->outer_mode = mode;
  return GH_OK;
}

int gh_set_interface(gh_ctx* c, int mode) {
  if (!c) return GH_ERR_ARG;
  if (!c->have_domain) return fail(c, GH_ERR_ORDER, "gh_set_domain has not been called");
  if (mode != 0 && mode != 1) return fail(c, GH_ERR_ARG, "mode must be 0 (background) or 1 (state)");
  HIPCHK(c, hipSetDevice(c->device));
  int rc;
  if (mode == 1 && !c->d_bctab_s) {
    if ((rc = dalloc(c, &c->d_bctab_s, size_t(std::max(c->bc_total, 1))))) return rc;
    if ((rc = dalloc(c, &c->d_exscr, size_t(c->n_shells) * c->max_S))) return rc;
  }
  if (mode != c->iface_mode) drop_graph(c);
  c->iface_mode = mode;
  return GH_OK;
}

int gh_filter(gh_ctx* c, const double* u, double* out) {
  if (!c || !u || !out) return GH_ERR_ARG;
  if (!c->have_domain) return fail(c, GH_ERR_ORDER, "gh_set_domain has not been called");
  if (c->filter_kind == 0) return fail(c, GH_ERR_ARG, "the domain has no filter (filter_kind 0)");
  if (u == out) return fail(c, GH_ERR_ARG, "out must not be u");
  HIPCHK(c, hipSetDevice(c->device));
  return queue_filter(c, u, out);
}

int gh_tensor_filter_matrix(int L, int kind, const double* params, int transpose, long long* nnz,
                            long long* row_ptr, int* col, double* val) {
  if (L < 1 || L > 63 || (kind != 2 && kind != 3) || !params || !nnz) return GH_ERR_ARG;
  if ((kind == 2 && (!(params[0] >= 0.0 && params[0] < 1.0) || !(params[1] >= 0.0) || !(params[2] > 0.0))) ||
      (kind == 3 && !(params[0] >= 0.0)))
    return GH_ERR_ARG;
  const ghtf::Csr m = ghtf::coupling_matrix(L, kind, params, transpose != 0);
  const long long n = m.row_ptr.back();
  if (!row_ptr && !col && !val) {
    *nnz = n;
    return GH_OK;
  }
  if (!row_ptr || !col || !val || *nnz < n) return GH_ERR_ARG;
  std::copy(m.row_ptr.begin(), m.row_ptr.end(), row_ptr);
  std::copy(m.col.begin(), m.col.end(), col);
  std::copy(m.val.begin(), m.val.end(), val);
  *nnz = n;
  return GH_OK;
}

int gh_query(const gh_ctx* c, int what, long long* value) {
  if (!c || !value) return GH_ERR_ARG;
  if (!c->have_domain) return GH_ERR_ORDER;
  int bm = 0, bn = 0;
  switch (what) {
    case 0: ghk::tile_dims(c->deriv.shape, &bm, &bn); *value = bm * 1000LL + bn; break;
    case 1:
      if (c->filter_kind == 1) { ghk::tile_dims(c->filter.shape, &bm, &bn); *value = bm * 1000LL + bn; }
      else *value = 0;
      break;
    case 2: *value = c->deriv.n_tiles; break;
    case 3: *value = c->P; break;
    case 4: *value = c->deriv.order; break;
    case 5: *value = c->filter_kind == 1 ? c->filter.order : 0; break;
    case 6: *value = c->deriv.shape; break;
    case 7: *value = c->filter_kind == 1 ? c->filter.shape : -1; break;
    case 8: *value = c->ang_method; break;
    case 9: *value = c->deriv_tr ? 1 : 0; break;
    case 10: *value = c->filt_tr ? 1 : 0; break;
    case 11: *value = c->tf_nnz; break;
    case 12: *value = c->n_tf_items[0] + c->n_tf_items[1] + c->n_tf_items[2]; break;
    case 13: *value = c->iface_mode; break;
    case 17: *value = c->outer_mode; break;
    case 14: *value = c->deriv.n_ttiles ? c->deriv.tail_shape : -1; break;
    case 15: *value = c->filter.n_ttiles ? c->filter.tail_shape : -1; break;
    case 16: *value = c->deriv.n_ttiles ? c->deriv.tail_chunks : 0; break;
    default: return GH_ERR_ARG;
  }
  return GH_OK;
}

int gh_set_timing(gh_ctx* c, int enable) {
  if (!c) return GH_ERR_ARG;
  HIPCHK(c, hipSetDevice(c->device));
  if (c->stream) HIPCHK(c, hipStreamSynchronize(c->stream));
  if (enable < 0 || enable > 2) return fail(c, GH_ERR_ARG, "enable must be 0, 1 or 2");
  clear_timing(c);
  c->timing = enable != 0;
  c->timing_only = enable == 2 ? 0 : -1;
  return GH_OK;
}

int gh_kernel_stats(gh_ctx* c, int kind, long long* launches, double* total_ms) {
  if (!c || !launches || !total_ms || kind < 0 || kind >= GH_NUM_KERNEL_KINDS) return GH_ERR_ARG;
  HIPCHK(c, hipSetDevice(c->device));
  long long n = 0;
  double ms = 0.0;
  std::vector<gh_ctx::Rec> keep;
  for (auto& r : c->recs) {
    if (r.kind != kind) { keep.push_back(r); continue; }
    HIPCHK(c, hipEventSynchronize(r.b));
    float t = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&t, r.a, r.b));
    ms += t;
    ++n;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  c->recs.swap(keep);
  *launches = n;
  *total_ms = ms;
  return GH_OK;
}

int gh_grid_coords(int n_shells, const gh_shell* shells, double* xyz) {
  if (n_shells <= 0 || !shells || !xyz) return GH_ERR_ARG;
  long long P = 0;
  for (int k = 0; k < n_shells; ++k) {
    if (shells[k].n_r < 2 || shells[k].L < 0) return GH_ERR_ARG;
    P += (long long)shells[k].n_r * 2 * (shells[k].L + 1) * (shells[k].L + 1);
  }
  long long p = 0;
  for (int k = 0; k < n_shells; ++k) {
    const gh_shell& s = shells[k];
    auto xi = ghsetup::cgl_nodes(s.n_r);
    auto ang = ghsetup::angular_table(s.L);
    int S = 2 * (s.L + 1) * (s.L + 1);
    for (int j = 0; j < s.n_r; ++j) {
      double r = 0.5 * (s.r_in + s.r_out) + 0.5 * (s.r_out - s.r_in) * xi[j];
      for (int a = 0; a < S; ++a, ++p) {
        const double* t = &ang[size_t(a) * 5];
        xyz[p] = r * t[0] * t[3];
        xyz[P + p] = r * t[0] * t[2];
        xyz[2 * P + p] = r * t[1];
      }
    }
  }
  return GH_OK;
}

int gh_host_operator(int kind, int n, const double* params, double* out) {
  if (!out) return GH_ERR_ARG;
  if (kind >= 1 && kind <= 7 && kind != 4 && kind != 5 && n > 63) return GH_ERR_ARG;
  std::vector<double> v;
  switch (kind) {
    case 0: if (n < 2) return GH_ERR_ARG; v = ghsetup::cgl_diff_matrix(n); break;
    case 1: if (n < 1) return GH_ERR_ARG; v = ghsetup::sphere_operator(n, 0, {}); break;
    case 2: if (n < 1) return GH_ERR_ARG; v = ghsetup::sphere_operator(n, 1, {}); break;
    case 3:
      if (n < 1 || !params) return GH_ERR_ARG;
      v = ghsetup::sphere_operator(n, 2, ghsetup::exp_filter_sigma(n, params[0], params[1], params[2]));
      break;
    case 4: if (n < 2) return GH_ERR_ARG; v = ghsetup::clenshaw_curtis(n); break;
    case 6: {
      // the derivative GEMM's B operand (Theta^T | Phi^T), S x 2S, as uploaded
      if (n < 1) return GH_ERR_ARG;
      const size_t S = size_t(2) * (n + 1) * (n + 1);
      v.assign(S * 2 * S, 0.0);
      ghsetup::sphere_operator_into(n, 0, {}, true, v.data(), 2 * S);
      ghsetup::sphere_operator_into(n, 1, {}, true, v.data() + S, 2 * S);
      break;
    }
    case 7: {
      // the filter GEMM's B operand F^T, S x S, as uploaded
      if (n < 1 || !params) return GH_ERR_ARG;
      const size_t S = size_t(2) * (n + 1) * (n + 1);
      v.assign(S * S, 0.0);
      ghsetup::sphere_operator_into(n, 2, ghsetup::exp_filter_sigma(n, params[0], params[1], params[2]), true,
                                    v.data(), S);
      break;
    }
    case 5: {
      if (n < 0) return GH_ERR_ARG;
      std::vector<double> x, w;
      ghsetup::gauss_legendre(n, x, w);
      v = x;
      v.insert(v.end(), w.begin(), w.end());
      break;
    }
    default: return GH_ERR_ARG;
  }
  std::memcpy(out, v.data(), v.size() * sizeof(double));
  return GH_OK;
}

}  // extern "C"

int gh_step_dp5(gh_ctx* c, double* u, int n_attempts, double atol, double rtol, double* t, double* dt,
                int* rejected, int* n_accepted, double* err) {
  if (!c) return GH_ERR_ARG;
  if (!c->have_domain) return fail(c, GH_ERR_ORDER, "gh_set_domain has not been called");
  if (!c->have_bg) return fail(c, GH_ERR_ORDER, "gh_set_background has not been called");
  if (!c->have_gamma) return fail(c, GH_ERR_ORDER, "gh_set_params has not been called");
  if (!u || !t || !dt || n_attempts < 0 || !(atol >= 0.0) || !(rtol >= 0.0) || !(atol + rtol > 0.0) ||
      !std::isfinite(atol) || !std::isfinite(rtol))
    return fail(c, GH_ERR_ARG, "need device u, t, dt, n_attempts >= 0, atol, rtol >= 0 finite, atol + rtol > 0");
  HIPCHK(c, hipSetDevice(c->device));
  int rc = ensure_dp5(c);
  if (rc) return rc;
  if (n_attempts == 0) return GH_OK;
  const size_t F50 = size_t(50) * c->P;
  double* K[7];
  for (int j = 0; j < 7; ++j) K[j] = c->d_dpk + j * F50;
  const bool filt = c->filter_kind != 0;
  int* rej = rejected;
  if (!rej) {
    rej = c->d_dprej;
    HIPCHK(c, ghk::fill_int(rej, c->n_inst, 0, c->stream));
  }
  for (int a = 0; a < n_attempts; ++a) {
    // first stage: at the call's start, and after every filtered step (the
    // filtered state is not the last stage's), else the last stage's value
    if (a == 0 || filt)
      if ((rc = queue_rhs(c, u, K[0]))) return rc;
    for (int i = 1; i < 7; ++i) {
      double coef[7] = {0, 0, 0, 0, 0, 0, 0};
      for (int j = 0; j < i; ++j) coef[j] = dp5c::A[i][j];
      double* y = (i == 6) ? c->d_dpu5 : c->d_dpy;
      HIPCHK(c, ghk::dp_combine(c->d_sh, c->d_blk, c->n_blk, dt, u, K, coef, i, y, c->stream));
      if ((rc = queue_rhs(c, y, K[i]))) return rc;
    }
    HIPCHK(c, ghk::dp_error(c->d_sh, c->d_blk, c->n_blk, dt, u, c->d_dpu5, K, dp5c::E, atol, rtol, c->d_partial,
                            c->stream));
    HIPCHK(c, ghk::dp_control(c->d_inst_range, c->n_inst, c->d_dpnval, c->d_partial, dt, t, rej, c->d_dpacc,
                              n_accepted, err, c->stream));
    if (filt) {
      if ((rc = queue_filter(c, c->d_dpu5, c->d_dpf))) return rc;
      HIPCHK(c, ghk::dp_accept(c->d_sh, c->d_blk, c->n_blk, c->d_dpacc, c->d_dpf, u, nullptr, nullptr, c->stream));
    } else {
      HIPCHK(c, ghk::dp_accept(c->d_sh, c->d_blk, c->n_blk, c->d_dpacc, c->d_dpu5, u, K[6], K[0], c->stream));
    }
  }
  return GH_OK;
}
