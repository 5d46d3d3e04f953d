// Host runtime of libmabd: validation, topology classification, solve
// schedules, device buffers and the per-step launch sequence behind the C ABI
// declared in include/mabd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mabd.h"
#include "common.hpp"
#include "generic.hpp"
#include "gnn.hpp"

namespace mabd {

void launch_chain_reduce(const ChainArgs &a, int ntiles, int nt, bool pack, int mode,
                         hipStream_t s);
void launch_chain_apply(const ChainArgs &a, int ntiles, int nt, bool pack, int mode,
                        hipStream_t s);
void launch_chain_global(const ChainDesc *chains, int nchains, const double *tilerec, double *scr,
                         double *xg, uint32_t *status, int step, const double *ir, hipStream_t s);
void launch_chain_group(bool apply, const ChainDesc *chains, const GroupDesc *groups, int ngroups,
                        const double *tilerec, double *grouprec, double *xtop, double *xg,
                        double *gfac, int *counters, uint32_t *status, int step, const double *ir,
                        hipStream_t s);
void launch_chain_resid(const ChainArgs &a, int ntiles, int nt, hipStream_t s);
void launch_chain_ir_check(const double *part, int nblk, double tol, int final_check, double *ir,
                           uint32_t *status, hipStream_t s);
void launch_chain_ir_reset(double *ir, hipStream_t s);
void launch_chain_finish(const double *q, const double *dq, double *q_out, double *qd_out, int64_t ns,
                         int nb, double h, uint32_t *status, hipStream_t s);
void launch_prefactor(const double *shape, int nshape, double h, double *hinv, hipStream_t s);
void launch_gbody(int b0, int b1, const double *q, const double *qn, const double *qdn, int64_t ns,
                  const int32_t *shp, const double *hinv, const double *shape, const double *g,
                  double h, double *Rg, double *ug, uint32_t *status, int step, const double *wr,
                  const int32_t *pf_inc, int f32, const int32_t *free_inc, double *q_out, double *qd_out,
                  int acc, double *dq_save, hipStream_t s);
void launch_lam_add(int64_t n, double *glam, const double *dlam, const uint32_t *status, hipStream_t s);
void launch_raise(uint32_t *status, uint32_t flag, hipStream_t s);
void launch_gjoint(int m, const GJoint *J, const double *q, const double *Rg, int64_t ns, int hg,
                   double *gl, hipStream_t s);
void launch_tree(const TreeArgs &a, const GJoint *J, int nslots, const int32_t *rounds, int nround,
                 int split_ops, int order, const PathPlan *path, hipStream_t s, int hook_round = -1,
                 void (*hook)(void *) = nullptr, void *hook_arg = nullptr);
void launch_path(const TreeArgs &a, const PathPlan &P, hipStream_t s);
void launch_gapply(int b0, int b1, const int32_t *inc_off, const int32_t *inc, const double *gl,
                   const double *glam, const double *Rg, const double *ug, int64_t ns,
                   const int32_t *shp, const double *hinv, const double *q_cur, double *q_out,
                   double *qd_out, double h, int acc, uint32_t *status, const uint8_t *jrows,
                   int step, double *dq_save, int polar_free, int skip_free, hipStream_t s);
void launch_gather_state(int nd, const int32_t *sol2in, const double *const *q, const double *const *qd,
                         int cur, int cur0, const uint32_t *status, int64_t ns, double *qo, double *qdo,
                         hipStream_t s);
int diag_body_blocks(int nb);
void launch_gdiag_body(int b0, int b1, const double *q, const double *qn, const double *qdn,
                       const double *dqv, double dq_scale, int64_t ns, const int32_t *shp,
                       const double *hinv, const double *shape, const double *g, double h,
                       const double *Rg, const int32_t *inc_off, const int32_t *inc, const GJoint *J,
                       const double *gl, const double *glam, const double *wr, const uint32_t *status,
                       double *part, int polar_free, double *ucorr, hipStream_t s);
void launch_gdiag_joint(int m, const GJoint *J, const double *gl, const double *Rg, const double *ug,
                        const double *dqv, double dq_scale, const double *q_new, int64_t ns,
                        const uint32_t *status, double *part, double *ccorr, hipStream_t s);
void launch_diag_reduce(const double *part, int nblk, double *out, const uint32_t *status,
                        hipStream_t s);
int resid_static_blocks();
hipError_t resid_scratch(int device, double **out);
void launch_loop_inject(int nloop, const int32_t *loff, const int32_t *lrow, int j, const GJoint *J,
                        const double *gl, const int32_t *shp, const double *hinv, int64_t ns, double *uloop,
                        int set, hipStream_t s);
void launch_loop_schur(int nloop, const int32_t *loff, const int32_t *lrow, const GJoint *J, const double *gl,
                       const double *ug, const int32_t *shp, const double *hinv, int64_t ns,
                       const int32_t *inc_off, const int32_t *inc, const int32_t *jloop, const double *wcol,
                       int64_t wstride, double *glam, double *lamD, uint32_t *status, hipStream_t s);
void launch_loop_correct(int mj, const int32_t *jloop, const int32_t *loff, const double *wcol, int64_t wstride,
                         const double *lamD, double *glam, const uint32_t *status, hipStream_t s);
void launch_twists(int nd, const int32_t *sol2in, const double *q, const double *qd, int64_t ns,
                   double *V, hipStream_t s);
void launch_joint_wrenches(const ChainDesc *chains, int nchains, int nchain_bodies, const double *pl,
                           const double *pr, const uint8_t *flag, int64_t nrs, const double *clam,
                           int b0, int b1, const double *Rg, const int32_t *inc_off, const int32_t *inc,
                           const GJoint *J, const double *gl, const double *glam, const double *q,
                           int64_t ns, const int32_t *sol2in, double *W, hipStream_t s);
void launch_scatter_state(int nd, const int32_t *sol2in, const double *qi, const double *qdi,
                          double *q, double *qd, int64_t ns, hipStream_t s);
void launch_write_pinned(int np, const int32_t *idx, const double *q0, double *qo, double *qdo,
                         hipStream_t s);
void launch_reset_status(uint32_t *status, hipStream_t s);
void launch_begin_step(uint32_t *status, hipStream_t s);
hipError_t launch_pcg(const PcgArgs &a, int nblocks, hipStream_t s);
void launch_pb_setup(const PcgBallArgs &a, hipStream_t s);
void launch_pb_residual(const PcgBallArgs &a, int use_x, int verify, hipStream_t s);
void launch_pb_iters(const PcgBallArgs &a, int n, int first, hipStream_t s);
void launch_pb_finish(const PcgBallArgs &a, hipStream_t s);
void launch_gnn_forward(const PcgBallArgs &a, const GnnBufs &g, int have_prev, hipStream_t s);
void launch_gnn_loss(const PcgBallArgs &a, const GnnBufs &g, hipStream_t s);
void launch_gnn_backward(const PcgBallArgs &a, const GnnBufs &g, hipStream_t s);
void launch_gnn_adam(const GnnBufs &g, float lr, int64_t t, hipStream_t s);
void launch_gnn_add_base(const PcgBallArgs &a, const GnnBufs &g, hipStream_t s);
int gnn_wgrad_blocks(int nj);
int pcg_max_blocks();
}  // namespace mabd

using namespace mabd;

namespace {

std::string g_create_error;

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

enum Cls { CLS_CHAIN = 1, CLS_TREE = 2, CLS_GRAPH = 3, CLS_LOOP = 4 };

// ------------------------------------------------------------ host 3x3 help
void polar_host(const double *A, double *R) {
  double X[9];
  std::memcpy(X, A, sizeof X);
  for (int it = 0; it < 60; ++it) {
    double C[9] = {X[4] * X[8] - X[5] * X[7], X[5] * X[6] - X[3] * X[8], X[3] * X[7] - X[4] * X[6],
                   X[2] * X[7] - X[1] * X[8], X[0] * X[8] - X[2] * X[6], X[1] * X[6] - X[0] * X[7],
                   X[1] * X[5] - X[2] * X[4], X[2] * X[3] - X[0] * X[5], X[0] * X[4] - X[1] * X[3]};
    double det = X[0] * C[0] + X[1] * C[1] + X[2] * C[2];
    double z = std::cbrt(1.0 / det), diff = 0.0;
    for (int i = 0; i < 9; ++i) {
      double xn = 0.5 * (z * X[i] + C[i] / (det * z));
      diff += (xn - X[i]) * (xn - X[i]);
      X[i] = xn;
    }
    if (diff < 1e-30) break;
  }
  std::memcpy(R, X, sizeof X);
}

void hinge_rod(const double *a, double *Rh) {
  // rows (r_x, a, r_z): the rotation taking the unit axis a to e_y (Sec. 4.3)
  if (1.0 + a[1] < 1e-12) {
    const double D[9] = {1, 0, 0, 0, -1, 0, 0, 0, -1};
    std::memcpy(Rh, D, sizeof D);
    return;
  }
  const double v[3] = {-a[2], 0.0, a[0]};  // a x e_y
  const double K[9] = {0, -v[2], v[1], v[2], 0, -v[0], -v[1], v[0], 0};
  double K2[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      K2[3 * r + c] = K[3 * r] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
  for (int i = 0; i < 9; ++i) Rh[i] = (i % 4 == 0 ? 1.0 : 0.0) + K[i] + K2[i] / (1.0 + a[1]);
}

void mat3_vec_h(const double *A, const double *x, double *y) {
  for (int r = 0; r < 3; ++r) y[r] = A[3 * r] * x[0] + A[3 * r + 1] * x[1] + A[3 * r + 2] * x[2];
}
void mat3t_vec_h(const double *A, const double *x, double *y) {
  for (int r = 0; r < 3; ++r) y[r] = A[r] * x[0] + A[3 + r] * x[1] + A[6 + r] * x[2];
}

int find(std::vector<int> &p, int x) {
  while (p[x] != x) x = p[x] = p[p[x]];
  return x;
}

}  // namespace

struct mabd_ctx {
  std::string err;
  mabd_options opt;
  int n = 0, m = 0;
  // host copies
  std::vector<double> q0_in, qd0_in;
  std::vector<uint8_t> pinned;
  std::vector<uint8_t> jtype;
  std::vector<int32_t> jrow_off;  // input joint -> row offset in the input-order lambda
  int64_t nrows_total = 0;
  // solver order
  int nd = 0;
  int64_t ns = 0;
  std::vector<int32_t> sol2in, in2sol;
  std::vector<int32_t> pin_idx;
  // shapes
  int nshape = 0;
  // chains
  std::vector<ChainDesc> chains;
  std::vector<TileDesc> tiles;
  std::vector<GroupDesc> groups;
  int nchain_rows = 0, nchain_bodies = 0, ngrows = 0, ntop = 0;
  std::vector<int32_t> crow_joint;  // chain row -> input joint
  // generic
  std::vector<GJoint> gj;
  std::vector<int32_t> gj_in;
  int gb0 = 0, gb1 = 0;
  int ntree = 0, ngraph = 0;
  // components with a few loops (loop-breaker Schur complement): per generic
  // joint its loop component (-1 none, -2 a loop-closing joint), per
  // component its loop rows (joint << 3 | row), the columns S_AA^{-1} S_AD
  // (loop_maxr of 5 per generic joint), l_D, and the zero-based increments
  // of the column solves
  int nloop = 0, loop_maxr = 0;
  std::vector<int32_t> jloop, loff{0}, lrow;
  int32_t *d_jloop = nullptr, *d_loff = nullptr, *d_lrow = nullptr;
  double *d_wcol = nullptr, *d_lamD = nullptr, *d_uloop = nullptr;
  std::vector<int32_t> comp_lvl, lvl_off, tbody, tpk, tabs_off, tabs, inc_off, inc, tne;
  std::vector<int64_t> foff;
  int64_t fac_size = 0;
  // tree contraction schedule
  std::vector<TcOp> tc_ops;
  std::vector<int32_t> tc_rounds;  // TC_NSEG * rounds + 1 offsets into tc_ops (segments by kind and size)
  int64_t crec_size = 0;
  TcOp *d_tc_ops = nullptr;
  double *d_crec = nullptr;
  // paths: tree components whose bodies carry at most two joints, solved as
  // block-tridiagonal systems over their joints (segments of path_T units
  // per lane, level by level); per path its input joints in path order and
  // the dynamic bodies before and after each (-1: none)
  // segment lengths: 16 units per lane at level 0; 4 above, where the few
  // separators leave the lanes' dependent steps, not memory, as the bound
  int npath = 0, path_T = 16, path_T1 = 4;
  std::vector<std::vector<int>> path_j, path_bb, path_ba;
  PathPlan pplan{};
  std::vector<PathUnitF> pu0;
  // with both paths (at least 16,384 joints) and contracted trees: the
  // step's path solve runs on a second stream beside the contraction rounds
  // (forked and joined by events)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int fork_round = 0;  // forward round of the contraction before which the paths fork
  std::vector<PathSeg> pseg;
  std::vector<int32_t> prows;
  int32_t *d_tne = nullptr;
  int64_t *d_foff = nullptr;
  double *d_fac = nullptr;
  // device
  std::vector<void *> allocs;
  double *d_q[2] = {nullptr, nullptr}, *d_qd[2] = {nullptr, nullptr};
  int cur = 0;
  int32_t *d_shp = nullptr;
  double *d_shape = nullptr, *d_hinv = nullptr;
  ChainDesc *d_chains = nullptr;
  TileDesc *d_tiles = nullptr;
  GroupDesc *d_groups = nullptr;
  double *d_grouprec = nullptr, *d_xtop = nullptr;
  double *d_gfac = nullptr;  // factors of the group reductions, PACK_CF x CHAIN_THREADS per group
  int *d_gcount = nullptr;
  int tile_threads = 64;     // workgroup size of the chain tile kernels (autotuned)
  bool tile_pack = true;     // packed 64-thread tiles (autotuned)
  // packed tiles, per group of four tiles: survivors and factors
  double *d_psv = nullptr, *d_pcf = nullptr;
  bool top_in_group = true;  // every chain's top system fits one workgroup
  // MABD_CHAIN_TOP_GLOBAL=1: every chain's top system goes through
  // chain_global_kernel (the path of chains beyond ~3.9M rows), for testing
  bool force_top_global = false;
  bool tuned = false;
  // tree contraction schedule (autotuned): a round's 16-row classes launch
  // apart when they hold more than tree_split operations; class order within
  // a launch, 0 largest cliques first, 1 smallest first
  int tree_split = 6000;
  int tree_order = 0;
  int tune_source = 0;     // 0 defaults, 1 timed, 2 read from the tuning cache
  // precision form 1 on the generic components (trees): FP32 local solves
  // and clique assembly, FP64 factor, host-controlled FP64 refinement
  bool gen_ir = false;
  double *d_uc = nullptr, *d_cc = nullptr, *d_dlam = nullptr;  // correction rhs, multipliers
  double *d_irpart = nullptr, *d_irout = nullptr, *h_irout = nullptr;
  int gir_sweeps = 0, gir_stalled = 0;
  double gir_rho_p = -1.0, gir_rho_d = -1.0, gir_kkt = -1.0;
  std::string tune_cache;  // path of the tuning cache file ("" none)
  // captured step graphs, one per state-buffer parity
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  // external wrenches: 6 x ns doubles (solver order, SoA), used while wr_on
  double *d_wr = nullptr;
  bool wr_on = false;
  bool graph_failed = false;
  double *d_pl = nullptr, *d_pr = nullptr;
  uint8_t *d_flag = nullptr;
  double *d_tilerec = nullptr, *d_grow = nullptr, *d_xg = nullptr, *d_clam = nullptr;
  GJoint *d_gj = nullptr;
  uint8_t *d_jrows = nullptr;  // rows per generic joint
  double *d_gl = nullptr, *d_gt = nullptr, *d_glam = nullptr, *d_Rg = nullptr, *d_ug = nullptr;
  int32_t *d_comp_lvl = nullptr, *d_lvl_off = nullptr, *d_tbody = nullptr, *d_tpk = nullptr,
          *d_tabs_off = nullptr, *d_tabs = nullptr, *d_inc_off = nullptr, *d_inc = nullptr;
  int32_t *d_sol2in = nullptr, *d_pin_idx = nullptr;
  // graph components (PCG)
  std::vector<int32_t> jmask, bmask;
  int32_t *d_jmask = nullptr, *d_bmask = nullptr;
  double *d_pbv = nullptr;
  double *d_pr_ = nullptr, *d_pp = nullptr, *d_pz = nullptr, *d_psp = nullptr, *d_dinv = nullptr,
         *d_zb = nullptr, *d_partial = nullptr, *d_pcg_res = nullptr;
  int32_t *d_pcg_it = nullptr;
  int pcg_blocks = 0;
  // compact operator when every graph joint is a ball joint
  bool pcg_ball = false;
  int pb_nj = 0, pb_nbd = 0, pb_blocks = 0;
  int32_t *d_pb_jid = nullptr, *d_pb_jba = nullptr, *d_pb_jbb = nullptr, *d_pb_bid = nullptr,
          *d_pb_boff = nullptr, *d_pb_binc = nullptr;
  double *d_pb_jp = nullptr, *d_pb_vec = nullptr, *d_pb_dinv = nullptr, *d_pb_zw = nullptr,
         *d_pb_sc = nullptr;
  int32_t *d_pb_si = nullptr, *h_pb_si = nullptr;
  // learned warm start (allocated by mabd_gnn_init / mabd_gnn_load)
  bool gnn_ready = false;
  GnnBufs gb{};
  int64_t gnn_t = 0;       // Adam steps taken
  double *h_gsc = nullptr;  // pinned copies of loss / energy
  double *h_pcg = nullptr;
  // precision form 1 on the chains
  double *d_dq = nullptr, *d_rp = nullptr, *d_rd = nullptr, *d_part = nullptr, *d_ir = nullptr;
  double *h_ir = nullptr;
  double *d_pin_q0 = nullptr, *d_tmp = nullptr;
  uint32_t *d_status = nullptr;
  uint32_t *h_status = nullptr;
  // status of issued steps not read yet (mabd_step is asynchronous): the
  // state buffer current when the status word was cleared, the steps issued
  // since then, and an event recorded after the status copies
  bool pending = false;
  int pend_cur0 = 0;
  int64_t pend_steps = 0;
  hipEvent_t pend_ev = nullptr;
  // step diagnostics: DIAG_PART partial records (diag_nblk of them), the
  // reduced values {rho_p, rho_d, kkt, c_ball, c_hinge} of the step and of
  // each Newton iteration, their pinned host copy, and the iterate and
  // increment of the running Newton iteration
  double *d_dpart = nullptr, *d_diag = nullptr, *h_diag = nullptr;
  double *d_qit = nullptr, *d_dqit = nullptr;
  bool resid_ok = false;  // the buffers still describe the last completed step
  // this device's copy of the library's fixed residual scratch (not owned)
  double *d_rscratch = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  double h_last = -1.0;
  bool warm_valid = false;
  mabd_step_stats stats{};
  // kernel-group timing (diagnostics bit 1)
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_marks;  // (phase, index of the start event)
};

namespace {

mabd_status fail(mabd_ctx *c, mabd_status st, const std::string &msg) {
  if (c) c->err = msg;
  else g_create_error = msg;
  return st;
}

mabd_status resolve(mabd_ctx *c);

// reduced diagnostics per context: the step's five values, then five per
// Newton iteration (at most MABD_NEWTON_DIAG iterations are recorded)
constexpr int DIAG_VALUES = 5 * (1 + MABD_NEWTON_DIAG);

// partial records of one residual evaluation: chain tiles, then blocks of
// generic bodies, then blocks of generic joints
int64_t diag_nblk(const mabd_ctx *c) {
  return (int64_t)c->tiles.size() + diag_body_blocks(c->gb1 - c->gb0) + diag_body_blocks((int)c->gj.size());
}

template <typename T>
hipError_t dalloc(mabd_ctx *c, T **p, size_t count) {
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e == hipSuccess) {
    c->allocs.push_back(q);
    *p = static_cast<T *>(q);
  }
  return e;
}

// Sorts the operations of one round and kind, from ops[rounds.back()] to the
// end, into size classes (clique rows <= rows[k]) and appends the class ends
// to rounds (nclass values; larger cliques form a last class ending at
// ops.end(), the start of the next segment).  A class whose operations all fit at once into
// the next class's kernel (count <= cap[k + 1]) joins that class: one launch
// fewer on the critical path of a small round.
template <class Size>
void segment_ops(std::vector<TcOp> &ops, std::vector<int32_t> &rounds, Size size, const int *rows,
                 const int *cap, int nclass) {
  auto b = ops.begin() + rounds.back();
  auto cls = [&](const TcOp &o) {
    const int r = size(o);
    for (int k = 0; k < nclass; ++k)
      if (r <= rows[k]) return k;
    return nclass;
  };
  std::vector<int> cnt(nclass + 1, 0), up(nclass + 1);
  for (auto it = b; it != ops.end(); ++it) ++cnt[cls(*it)];
  for (int k = 0; k <= nclass; ++k) up[k] = k;
  for (int k = 0; k + 1 < nclass; ++k)
    if (cnt[k] > 0 && cnt[k] + cnt[k + 1] <= cap[k + 1]) {
      cnt[k + 1] += cnt[k];
      cnt[k] = 0;
      for (int q = 0; q <= k; ++q)
        if (up[q] == k) up[q] = k + 1;
    }
  std::stable_sort(b, ops.end(), [&](const TcOp &x, const TcOp &y) { return up[cls(x)] < up[cls(y)]; });
  for (int k = 0; k < nclass; ++k)
    rounds.push_back((int)(std::partition_point(b, ops.end(), [&](const TcOp &o) { return up[cls(o)] <= k; }) -
                           ops.begin()));
}

template <typename T>
hipError_t upload(mabd_ctx *c, T **p, const std::vector<T> &v) {
  hipError_t e = dalloc(c, p, v.size());
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

bool finite_all(const double *p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

namespace {
// time a group of launches with a pair of events when diagnostics bit 1 is set
struct PhaseTimer {
  mabd_ctx *c;
  bool on;
  size_t used = 0;
  PhaseTimer(mabd_ctx *cc) : c(cc), on((cc->opt.diagnostics & 2) != 0) { c->ev_marks.clear(); }
  hipEvent_t next() {
    if (used == c->ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) { on = false; return nullptr; }
      c->ev_pool.push_back(e);
    }
    return c->ev_pool[used++];
  }
  template <typename F>
  void run(int phase, F &&f) {
    if (!on) { f(); return; }
    hipEvent_t a = next(), b = next();
    if (!on) { f(); return; }
    (void)hipEventRecord(a, c->stream);
    f();
    (void)hipEventRecord(b, c->stream);
    c->ev_marks.emplace_back(phase, (int)used - 2);
  }
  void collect() {
    for (int i = 0; i < MABD_NPHASES; ++i) { c->stats.phase_ms[i] = 0.0; c->stats.phase_calls[i] = 0; }
    if (!on) return;
    for (auto &pm : c->ev_marks) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c->ev_pool[pm.second], c->ev_pool[pm.second + 1]) == hipSuccess) {
        c->stats.phase_ms[pm.first] += ms;
        c->stats.phase_calls[pm.first] += 1;
      }
    }
  }
};
}  // namespace

namespace {
bool tune_chain(const mabd_ctx *c);
bool tune_tree(const mabd_ctx *c);
bool tune_cache_read(const mabd_ctx *c, int &tt, int &pack, int &split, int &order);
}  // namespace

namespace {
// Tiles of tile_threads - 2 rows (PACK_T rows for packed tiles) and groups of
// GROUP_T + 1 interface rows for every chain; descriptors go to preallocated
// device buffers (sized for the smallest tiles), so re-tuning only rewrites
// them.
hipError_t build_tiles(mabd_ctx *c, int tt, bool pack) {
  if (pack) tt = 64;
  c->tile_threads = tt;
  c->tile_pack = pack;
  c->tiles.clear();
  c->groups.clear();
  c->ngrows = 0;
  c->ntop = 0;
  c->top_in_group = true;
  const int TT = pack ? PACK_T : tt - 2;
  for (size_t ci = 0; ci < c->chains.size(); ++ci) {
    ChainDesc &cd = c->chains[ci];
    const int K = cd.K;
    cd.ntile = (K - 1 + TT - 1) / TT;
    cd.tile0 = (int)c->tiles.size();
    cd.grow0 = c->ngrows;
    for (int t = 0; t < cd.ntile; ++t) {
      TileDesc td{};
      td.chain = (int)ci;
      td.r0 = t * TT;
      td.T = std::min(TT, K - 1 - td.r0);
      td.tidx = t;
      c->tiles.push_back(td);
    }
    c->ngrows += cd.ntile + 1;
    cd.ngroup = (cd.ntile + GROUP_T - 1) / GROUP_T;
    cd.group0 = (int)c->groups.size();
    cd.gtop0 = c->ntop;
    for (int g2 = 0; g2 < cd.ngroup; ++g2) {
      GroupDesc gd{};
      gd.chain = (int)ci;
      gd.g0 = g2 * GROUP_T;
      gd.T = std::min(GROUP_T, cd.ntile - gd.g0);
      gd.gidx = g2;
      c->groups.push_back(gd);
    }
    c->ntop += cd.ngroup + 1;
    cd.top_global = (cd.ngroup + 1 > CHAIN_THREADS || c->force_top_global) ? 1 : 0;
    if (cd.top_global) c->top_in_group = false;
  }
  if (!c->d_chains) return hipSuccess;  // not allocated yet (create sizes them first)
  hipError_t e = hipMemcpy(c->d_chains, c->chains.data(), c->chains.size() * sizeof(ChainDesc),
                           hipMemcpyHostToDevice);
  if (e == hipSuccess && !c->tiles.empty())
    e = hipMemcpy(c->d_tiles, c->tiles.data(), c->tiles.size() * sizeof(TileDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess && !c->groups.empty())
    e = hipMemcpy(c->d_groups, c->groups.data(), c->groups.size() * sizeof(GroupDesc),
                  hipMemcpyHostToDevice);
  return e;
}
}  // namespace

extern "C" {

void mabd_options_default(mabd_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->gravity[2] = -9.8;
  o->precision = 0;
  o->kkt_tol = 1e-10;
  o->max_iters = 200000;
  o->warm_start = 0;
  o->newton_iters = 1;
  o->hinge_grad = 0;
  o->material = 0;
  o->diagnostics = 0;
  o->use_graph = 1;
  o->autotune = 1;
  o->ir_max_sweeps = 4;
  o->body_solve = 0;
  o->path_solver = 1;
  o->tune_cache = nullptr;
  o->stream = nullptr;
}

const char *mabd_last_error(const mabd_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

void mabd_destroy(mabd_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (int i = 0; i < 2; ++i)
    if (c->gexec[i]) (void)hipGraphExecDestroy(c->gexec[i]);
  for (hipEvent_t ev : c->ev_pool) (void)hipEventDestroy(ev);
  for (void *p : c->allocs) (void)hipFree(p);
  if (c->h_status) (void)hipHostFree(c->h_status);
  if (c->h_pcg) (void)hipHostFree(c->h_pcg);
  if (c->h_ir) (void)hipHostFree(c->h_ir);
  if (c->h_pb_si) (void)hipHostFree(c->h_pb_si);
  if (c->h_gsc) (void)hipHostFree(c->h_gsc);
  if (c->h_diag) (void)hipHostFree(c->h_diag);
  if (c->h_irout) (void)hipHostFree(c->h_irout);
  if (c->pend_ev) (void)hipEventDestroy(c->pend_ev);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->side) (void)hipStreamDestroy(c->side);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

int64_t mabd_rows(const mabd_ctx *c) { return c ? c->nrows_total : 0; }

mabd_status mabd_create(const mabd_bodies *B, const mabd_joints *Jn, const mabd_options *o,
                        mabd_ctx **out) {
  g_create_error.clear();
  if (!out) return fail(nullptr, MABD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!B || B->n < 0) return fail(nullptr, MABD_ERR_INVALID_ARG, "bodies missing or n < 0");
  const int n = B->n;
  const int m = Jn ? Jn->m : 0;
  if (m < 0) return fail(nullptr, MABD_ERR_INVALID_ARG, "m < 0");
  if (n > 0 && (!B->dims || !B->density || !B->k_orth || !B->q0))
    return fail(nullptr, MABD_ERR_INVALID_ARG, "dims, density, k_orth and q0 are required");
  if (m > 0 && (!Jn->type || !Jn->a || !Jn->b || !Jn->pa || !Jn->pb))
    return fail(nullptr, MABD_ERR_INVALID_ARG, "joint type, a, b, pa, pb are required");
  mabd_options opt;
  if (o) opt = *o;
  else mabd_options_default(&opt);
  if (opt.newton_iters < 1) return fail(nullptr, MABD_ERR_INVALID_ARG, "newton_iters < 1");
  if (opt.material != 0 && opt.material != 1) return fail(nullptr, MABD_ERR_INVALID_ARG, "material");
  if (opt.material == 1 && n > 0 && !B->poisson)
    return fail(nullptr, MABD_ERR_INVALID_ARG, "material 1 needs poisson");
  if (opt.hinge_grad != 0 && opt.hinge_grad != 2)
    return fail(nullptr, MABD_ERR_INVALID_ARG, "hinge_grad must be 0 or 2");
  if (opt.warm_start < 0 || opt.warm_start > 2)
    return fail(nullptr, MABD_ERR_INVALID_ARG, "warm_start must be 0, 1 or 2");
  if (opt.precision != 0 && opt.precision != 1)
    return fail(nullptr, MABD_ERR_INVALID_ARG, "precision must be 0 or 1");
  if (opt.ir_max_sweeps < 0 || opt.ir_max_sweeps > 16)
    return fail(nullptr, MABD_ERR_INVALID_ARG, "ir_max_sweeps must be in 0..16");
  if (opt.body_solve != 0 && opt.body_solve != 1)
    return fail(nullptr, MABD_ERR_INVALID_ARG, "body_solve must be 0 or 1");
  if (opt.path_solver != 0 && opt.path_solver != 1)
    return fail(nullptr, MABD_ERR_INVALID_ARG, "path_solver must be 0 or 1");
  if (!finite_all(opt.gravity, 3)) return fail(nullptr, MABD_ERR_INVALID_ARG, "gravity not finite");
  // ------------------------------------------------------------ validate
  for (int i = 0; i < n; ++i) {
    const double *d = B->dims + 3 * i;
    if (!(d[0] > 0 && d[1] > 0 && d[2] > 0) || !std::isfinite(d[0] * d[1] * d[2]))
      return fail(nullptr, MABD_ERR_INVALID_ARG, "body " + std::to_string(i) + ": dims must be > 0");
    if (!(B->density[i] > 0) || !std::isfinite(B->density[i]))
      return fail(nullptr, MABD_ERR_INVALID_ARG, "body " + std::to_string(i) + ": density");
    if (!(B->k_orth[i] > 0) || !std::isfinite(B->k_orth[i]))
      return fail(nullptr, MABD_ERR_INVALID_ARG, "body " + std::to_string(i) + ": stiffness");
    if (opt.material == 1 && !(B->poisson[i] > -1.0 && B->poisson[i] < 0.5))
      return fail(nullptr, MABD_ERR_INVALID_ARG, "body " + std::to_string(i) + ": poisson");
  }
  if (!finite_all(B->q0, (size_t)12 * n) || (B->qd0 && !finite_all(B->qd0, (size_t)12 * n)))
    return fail(nullptr, MABD_ERR_INVALID_ARG, "initial state not finite");
  std::vector<uint8_t> pinned(n, 0);
  if (B->pinned)
    for (int i = 0; i < n; ++i) pinned[i] = B->pinned[i] ? 1 : 0;
  auto dyn = [&](int b) { return b >= 0 && !pinned[b]; };
  for (int i = 0; i < n; ++i) {
    const double *q = B->q0 + 12 * i;
    double A[9] = {q[0], q[3], q[6], q[1], q[4], q[7], q[2], q[5], q[8]};
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                 A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(det > 0)) return fail(nullptr, MABD_ERR_INVALID_ARG, "body " + std::to_string(i) + ": det A <= 0");
  }
  for (int k = 0; k < m; ++k) {
    const int a = Jn->a[k], b = Jn->b[k];
    const std::string jk = "joint " + std::to_string(k) + ": ";
    if (Jn->type[k] > 3) return fail(nullptr, MABD_ERR_INVALID_ARG, jk + "type must be 0, 1, 2 or 3");
    if (a < -1 || a >= n || b < -1 || b >= n) return fail(nullptr, MABD_ERR_INVALID_ARG, jk + "body index");
    if (a == b) return fail(nullptr, MABD_ERR_INVALID_ARG, jk + "a == b");
    if (!dyn(a) && !dyn(b)) return fail(nullptr, MABD_ERR_INVALID_ARG, jk + "no dynamic side");
    if (!finite_all(Jn->pa + 3 * k, 3) || !finite_all(Jn->pb + 3 * k, 3))
      return fail(nullptr, MABD_ERR_INVALID_ARG, jk + "anchor not finite");
    if (Jn->type[k] != 0) {
      if (!Jn->axis || !Jn->cp_len)
        return fail(nullptr, MABD_ERR_INVALID_ARG, jk + "hinge, universal and prismatic joints need axis, cp_len");
      const double *ax = Jn->axis + 3 * k;
      double nrm = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
      if (!(nrm > 1e-12) || !std::isfinite(nrm)) return fail(nullptr, MABD_ERR_INVALID_ARG, jk + "zero hinge axis");
      if (!(Jn->cp_len[k] > 0) || !std::isfinite(Jn->cp_len[k]))
        return fail(nullptr, MABD_ERR_INVALID_ARG, jk + "cp_len must be > 0");
      if (Jn->type[k] == 2) {
        if (!Jn->axis2) return fail(nullptr, MABD_ERR_INVALID_ARG, jk + "universal joint needs axis2");
        const double *a2 = Jn->axis2 + 3 * k;
        const double n2 = std::sqrt(a2[0] * a2[0] + a2[1] * a2[1] + a2[2] * a2[2]);
        if (!(n2 > 1e-12) || !std::isfinite(n2)) return fail(nullptr, MABD_ERR_INVALID_ARG, jk + "zero axis2");
        const double cs = (ax[0] * a2[0] + ax[1] * a2[1] + ax[2] * a2[2]) / (nrm * n2);
        if (!(std::fabs(cs) <= 1e-6))
          return fail(nullptr, MABD_ERR_INVALID_ARG, jk + "axis2 must be orthogonal to axis");
      }
    }
  }

  mabd_ctx *c = new mabd_ctx();
  c->opt = opt;
  if (opt.tune_cache) c->tune_cache = opt.tune_cache;
  c->opt.tune_cache = nullptr;  // the context keeps its own copy
  c->n = n;
  c->m = m;
  c->pinned = pinned;
  c->q0_in.assign(B->q0, B->q0 + (size_t)12 * n);
  c->qd0_in.assign((size_t)12 * n, 0.0);
  if (B->qd0) c->qd0_in.assign(B->qd0, B->qd0 + (size_t)12 * n);
  c->jtype.assign(Jn ? Jn->type : nullptr, Jn ? Jn->type + m : nullptr);
  c->jrow_off.resize(m + 1, 0);
  for (int k = 0; k < m; ++k) c->jrow_off[k + 1] = c->jrow_off[k] + joint_rows(c->jtype[k]);
  c->nrows_total = c->jrow_off[m];

  // ------------------------------------------------------------ components
  std::vector<int> par(n);
  std::iota(par.begin(), par.end(), 0);
  for (int k = 0; k < m; ++k) {
    const int a = Jn->a[k], b = Jn->b[k];
    if (dyn(a) && dyn(b)) {
      int x = find(par, a), y = find(par, b);
      if (x != y) par[x] = y;
    }
  }
  std::map<int, int> comp_id;
  std::vector<int> body_comp(n, -1);
  for (int i = 0; i < n; ++i)
    if (dyn(i)) {
      int r = find(par, i);
      auto it = comp_id.find(r);
      if (it == comp_id.end()) it = comp_id.emplace(r, (int)comp_id.size()).first;
      body_comp[i] = it->second;
    }
  const int ncomp = (int)comp_id.size();
  std::vector<std::vector<int>> cbodies(ncomp), cjoints(ncomp);
  for (int i = 0; i < n; ++i)
    if (body_comp[i] >= 0) cbodies[body_comp[i]].push_back(i);
  std::vector<std::vector<int>> binc(n);  // incident joints per dynamic body
  for (int k = 0; k < m; ++k) {
    const int a = Jn->a[k], b = Jn->b[k];
    int ci = dyn(a) ? body_comp[a] : body_comp[b];
    cjoints[ci].push_back(k);
    if (dyn(a)) binc[a].push_back(k);
    if (dyn(b)) binc[b].push_back(k);
  }
  std::vector<int> cls(ncomp);
  std::vector<uint8_t> is_loop_joint(m, 0);
  for (int ci = 0; ci < ncomp; ++ci) {
    long edges = 0;
    int maxdeg = 0;
    bool all_ball = true;
    for (int k : cjoints[ci]) {
      edges += (dyn(Jn->a[k]) ? 1 : 0) + (dyn(Jn->b[k]) ? 1 : 0);
      if (Jn->type[k] != 0) all_ball = false;
    }
    for (int b : cbodies[ci]) maxdeg = std::max<int>(maxdeg, (int)binc[b].size());
    const long nodes = (long)cbodies[ci].size() + (long)cjoints[ci].size();
    const bool acyclic = edges == nodes - 1;
    if (!acyclic) {
      // few loops: loop-breaker Schur complement (Case III) on a spanning
      // tree, when its loop-closing joints have at most LOOP_MAX_ROWS rows
      std::set<int> seen{cbodies[ci][0]}, used;
      std::vector<int> order{cbodies[ci][0]};
      for (size_t h = 0; h < order.size(); ++h)
        for (int k : binc[order[h]]) {
          const int o = Jn->a[k] == order[h] ? Jn->b[k] : Jn->a[k];
          if (!dyn(o) || seen.count(o)) continue;
          seen.insert(o);
          used.insert(k);
          order.push_back(o);
        }
      int rows_d = 0;
      std::vector<int> dk;
      for (int k : cjoints[ci])
        if (dyn(Jn->a[k]) && dyn(Jn->b[k]) && !used.count(k)) {
          rows_d += joint_rows(Jn->type[k]);
          dk.push_back(k);
        }
      cls[ci] = (rows_d > 0 && rows_d <= LOOP_MAX_ROWS) ? CLS_LOOP : CLS_GRAPH;
      if (cls[ci] == CLS_LOOP)
        for (int k : dk) is_loop_joint[k] = 1;
    }
    else if (all_ball && maxdeg <= 2 && cjoints[ci].size() >= 2 && opt.newton_iters == 1)
      cls[ci] = CLS_CHAIN;
    else cls[ci] = CLS_TREE;
  }

  // ------------------------------------------------------------ solver order
  c->in2sol.assign(n, -1);
  auto add_body = [&](int i) {
    c->in2sol[i] = (int)c->sol2in.size();
    c->sol2in.push_back(i);
  };
  // chains
  std::vector<double> pl, pr;
  std::vector<uint8_t> cflag;
  auto world_point = [&](int b, const double *p, double *w) {
    if (b < 0) { std::memcpy(w, p, 3 * sizeof(double)); return; }
    const double *q = B->q0 + 12 * b;
    for (int r = 0; r < 3; ++r) w[r] = q[r] * p[0] + q[3 + r] * p[1] + q[6 + r] * p[2] + q[9 + r];
  };
  for (int ci = 0; ci < ncomp; ++ci) {
    if (cls[ci] != CLS_CHAIN) continue;
    const auto &js = cjoints[ci];
    // dual degree of a joint: other joints at its dynamic bodies
    auto ddeg = [&](int k) {
      int d = 0;
      for (int b : {Jn->a[k], Jn->b[k]})
        if (dyn(b)) d += (int)binc[b].size() - 1;
      return d;
    };
    int start = js[0];
    for (int k : js)
      if (ddeg(k) <= 1) { start = k; break; }
    std::vector<int> rows;
    std::vector<int> shared;  // body between rows r and r+1
    int prev_body = -1, cur = start;
    std::vector<char> used(0);
    rows.push_back(cur);
    for (;;) {
      int nxt = -1, via = -1;
      for (int b : {Jn->a[cur], Jn->b[cur]}) {
        if (!dyn(b) || b == prev_body) continue;
        for (int k2 : binc[b])
          if (k2 != cur) { nxt = k2; via = b; }
      }
      if (nxt < 0) break;
      shared.push_back(via);
      rows.push_back(nxt);
      prev_body = via;
      cur = nxt;
    }
    const int K = (int)rows.size();
    // end bodies
    auto other_dyn = [&](int k, int not_b) {
      for (int b : {Jn->a[k], Jn->b[k]})
        if (dyn(b) && b != not_b) return b;
      return -1;
    };
    const int left_end = other_dyn(rows[0], K > 1 ? shared[0] : -1);
    const int right_end = other_dyn(rows[K - 1], K > 1 ? shared[K - 2] : left_end);
    ChainDesc cd{};
    cd.hl = left_end < 0 ? 1 : 0;
    cd.hr = right_end < 0 ? 1 : 0;
    cd.K = K;
    cd.nb = K - 1 + (1 - cd.hl) + (1 - cd.hr);
    cd.body0 = (int)c->sol2in.size();
    cd.row0 = c->nchain_rows;
    if (cd.nb != (int)cbodies[ci].size()) {
      delete c;
      return fail(nullptr, MABD_ERR_TOPOLOGY, "internal: chain walk mismatch");
    }
    if (!cd.hl) add_body(left_end);
    for (int b : shared) add_body(b);
    if (!cd.hr) add_body(right_end);
    // row data
    for (int r = 0; r < K; ++r) {
      const int k = rows[r];
      const int lb = r == 0 ? left_end : shared[r - 1];
      const int rb = r == K - 1 ? right_end : shared[r];
      const int a = Jn->a[k], b = Jn->b[k];
      // which side of the joint is the left / right end
      bool left_is_a = lb >= 0 ? (a == lb) : !dyn(a);
      bool right_is_a = rb >= 0 ? (a == rb) : !dyn(a);
      if (lb < 0 && rb < 0) left_is_a = !dyn(a);
      double wl[3], wr[3];
      const double *pa = Jn->pa + 3 * k, *pb = Jn->pb + 3 * k;
      if (lb >= 0) std::memcpy(wl, left_is_a ? pa : pb, sizeof wl);
      else world_point(left_is_a ? a : b, left_is_a ? pa : pb, wl);
      if (rb >= 0) std::memcpy(wr, right_is_a ? pa : pb, sizeof wr);
      else world_point(right_is_a ? a : b, right_is_a ? pa : pb, wr);
      for (int i = 0; i < 3; ++i) { pl.push_back(wl[i]); pr.push_back(wr[i]); }
      cflag.push_back((left_is_a ? 1 : 0) | (right_is_a ? 2 : 0));
      c->crow_joint.push_back(k);
    }
    c->nchain_rows += K;
    c->chains.push_back(cd);
  }
  c->nchain_bodies = (int)c->sol2in.size();
  if (const char *tg = std::getenv("MABD_CHAIN_TOP_GLOBAL")) c->force_top_global = std::atoi(tg) != 0;
  (void)build_tiles(c, 64, true);  // sizes every tile buffer for the smallest tiles
  // generic (tree) components
  c->gb0 = c->nchain_bodies;
  std::vector<int> gidx(m, -1);  // input joint -> generic joint
  std::vector<int32_t> gj_graph;
  for (int ci = 0; ci < ncomp; ++ci) {
    if (cls[ci] != CLS_TREE && cls[ci] != CLS_GRAPH && cls[ci] != CLS_LOOP) continue;
    for (int k : cjoints[ci]) {
      gidx[k] = (int)c->gj_in.size();
      c->gj_in.push_back(k);
      gj_graph.push_back(cls[ci] == CLS_GRAPH ? 1 : 0);
    }
  }
  // tree schedules: root, BFS, heights, level order
  c->comp_lvl.push_back(0);
  c->lvl_off.push_back(0);
  for (int ci = 0; ci < ncomp; ++ci) {
    if (cls[ci] != CLS_TREE && cls[ci] != CLS_LOOP) continue;
    const auto &bs = cbodies[ci];
    if (cjoints[ci].empty()) {
      // a body without joints: its step is the body solve and the update
      // alone, no elimination slot
      add_body(bs[0]);
      c->ntree++;
      continue;
    }
    // a path: every body carries at most two joints (a tree, so its joints
    // form one sequence, consecutive joints sharing a body).  Its bodies
    // take no tree slot: they go into the solver order along the path, and
    // the path solve forms its blocks from the joint rows
    bool is_path = opt.path_solver != 0 && cls[ci] == CLS_TREE;
    for (int b : bs)
      if (binc[b].size() > 2) is_path = false;
    if (is_path) {
      const auto &js = cjoints[ci];
      std::map<int, std::vector<int>> jadj;  // joints sharing a body
      for (int b : bs)
        if (binc[b].size() == 2) {
          jadj[binc[b][0]].push_back(binc[b][1]);
          jadj[binc[b][1]].push_back(binc[b][0]);
        }
      int start = js[0];
      for (int k : js)
        if (jadj[k].size() < 2) { start = k; break; }
      std::vector<int> seq{start};
      std::set<int> used{start};
      for (;;) {
        int nxt = -1;
        for (int k2 : jadj[seq.back()])
          if (!used.count(k2)) nxt = k2;
        if (nxt < 0) break;
        used.insert(nxt);
        seq.push_back(nxt);
      }
      auto shared = [&](int k1, int k2) {
        for (int s1 : {Jn->a[k1], Jn->b[k1]})
          if (dyn(s1) && (s1 == Jn->a[k2] || s1 == Jn->b[k2])) return s1;
        return -1;
      };
      auto other = [&](int k, int excl) {  // a dynamic side of k other than excl
        for (int s1 : {Jn->a[k], Jn->b[k]})
          if (dyn(s1) && s1 != excl) return s1;
        return -1;
      };
      const int M = (int)seq.size();
      std::vector<int> bb(M), ba(M);
      for (int i = 0; i < M; ++i) {
        if (M == 1) {
          bb[0] = dyn(Jn->a[seq[0]]) ? Jn->a[seq[0]] : -1;
          ba[0] = dyn(Jn->b[seq[0]]) ? Jn->b[seq[0]] : -1;
          break;
        }
        bb[i] = i > 0 ? shared(seq[i - 1], seq[i]) : other(seq[0], shared(seq[0], seq[1]));
        ba[i] = i < M - 1 ? shared(seq[i], seq[i + 1]) : other(seq[M - 1], shared(seq[M - 2], seq[M - 1]));
      }
      // bodies along the path
      int added = 0;
      if (bb[0] >= 0) { add_body(bb[0]); ++added; }
      for (int i = 0; i < M; ++i)
        if (ba[i] >= 0 && (i == M - 1 || ba[i] == bb[i + 1])) { add_body(ba[i]); ++added; }
      if ((int)seq.size() != (int)js.size() || added != (int)bs.size()) {
        delete c;
        return fail(nullptr, MABD_ERR_TOPOLOGY, "path component: joints do not form one sequence");
      }
      c->path_j.push_back(seq);
      c->path_bb.push_back(bb);
      c->path_ba.push_back(ba);
      c->npath++;
      c->ntree++;
      continue;
    }
    int root = bs[0];
    for (int b : bs) {
      bool has_unary = false;
      for (int k : binc[b])
        if (!dyn(Jn->a[k]) || !dyn(Jn->b[k])) has_unary = true;
      if (has_unary) { root = b; break; }
    }
    std::map<int, int> parent_joint;  // body -> joint to its parent
    std::vector<int> order{root};
    std::map<int, int> seen{{root, 1}};
    for (size_t h = 0; h < order.size(); ++h) {
      int b = order[h];
      for (int k : binc[b]) {
        if (is_loop_joint[k]) continue;  // loop breakers stay out of the tree
        int o = Jn->a[k] == b ? Jn->b[k] : Jn->a[k];
        if (!dyn(o) || seen.count(o)) continue;
        seen[o] = 1;
        parent_joint[o] = k;
        order.push_back(o);
      }
    }
    std::map<int, int> height;
    for (auto it = order.rbegin(); it != order.rend(); ++it) {
      int b = *it;
      int hgt = 0;
      for (int k : binc[b]) {
        int o = Jn->a[k] == b ? Jn->b[k] : Jn->a[k];
        if (dyn(o) && parent_joint.count(o) && parent_joint[o] == k) hgt = std::max(hgt, height[o] + 1);
      }
      height[b] = hgt;
    }
    int maxh = 0;
    for (int b : order) maxh = std::max(maxh, height[b]);
    std::vector<std::vector<int>> lv(maxh + 1);
    for (int b : order) lv[height[b]].push_back(b);
    for (auto &L : lv) {
      for (int b : L) {
        add_body(b);
        c->tbody.push_back(c->in2sol[b]);
        int pk = -1;
        if (parent_joint.count(b)) {
          int k = parent_joint[b];
          pk = (gidx[k] << 1) | (Jn->a[k] == b ? 0 : 1);
        }
        c->tpk.push_back(pk);
        c->tabs_off.push_back((int)c->tabs.size());
        int unary_rows = 0;
        for (int k : binc[b]) {
          if (parent_joint.count(b) && parent_joint[b] == k) continue;
          if (is_loop_joint[k]) continue;
          const int side = Jn->a[k] == b ? 0 : 1;
          const bool unary = !dyn(Jn->a[k]) || !dyn(Jn->b[k]);
          if (unary) unary_rows += joint_rows(Jn->type[k]);
          c->tabs.push_back(abs_pack(gidx[k], joint_rows(Jn->type[k]), side, unary ? 1 : 0));
        }
        int ne = 0;
        for (int e = c->tabs_off.back(); e < (int)c->tabs.size(); ++e) ne += abs_rows(c->tabs[e]);
        const int nr = ne + (pk >= 0 ? joint_rows(Jn->type[parent_joint[b]]) : 0);
        if (nr > TREE_KMAX) {
          delete c;
          return fail(nullptr, MABD_ERR_TOPOLOGY, "a tree body has more than 64 joint rows around it");
        }
        c->tne.push_back(ne);
        c->foff.push_back(c->fac_size);
        c->fac_size += (int64_t)nr * nr + nr + (nr > TREE_KLDS ? 24 * (int64_t)nr : 0);
        (void)unary_rows;
      }
      c->lvl_off.push_back((int)c->tbody.size());
    }
    c->comp_lvl.push_back((int)c->lvl_off.size() - 1);
    if (cls[ci] == CLS_LOOP) {
      // loop rows and the joint -> loop component map (generic indices)
      if (c->jloop.empty()) c->jloop.assign(c->gj_in.size(), -1);
      int nr = 0;
      for (int k : cjoints[ci]) {
        c->jloop[gidx[k]] = is_loop_joint[k] ? -2 : c->nloop;
        if (!is_loop_joint[k]) continue;
        for (int r = 0; r < joint_rows(Jn->type[k]); ++r) c->lrow.push_back((gidx[k] << 3) | r);
        nr += joint_rows(Jn->type[k]);
      }
      c->loff.push_back((int)c->lrow.size());
      c->loop_maxr = std::max(c->loop_maxr, nr);
      c->nloop++;
    } else {
      c->ntree++;
    }
  }
  c->tabs_off.push_back((int)c->tabs.size());
  // ---- tree contraction schedule: rounds of rakes (slots with no live
  // child) and compresses (slots with exactly one live child, an independent
  // set chosen top-down), until every slot is eliminated
  {
    const int nsl = (int)c->tbody.size();
    std::vector<int> slot_of(c->sol2in.size(), -1);
    for (int s = 0; s < nsl; ++s) slot_of[c->tbody[s]] = s;
    std::vector<int> par(nsl, -1), kcur(nsl, -1), ckcur(nsl, 0), depth(nsl, 0);
    std::vector<std::vector<int>> kids(nsl);
    for (int s = 0; s < nsl; ++s) {
      const int pk = c->tpk[s];
      if (pk < 0) continue;
      const int kin = c->gj_in[pk >> 1];
      const int me = c->sol2in[c->tbody[s]];
      const int other = Jn->a[kin] == me ? Jn->b[kin] : Jn->a[kin];
      par[s] = slot_of[c->in2sol[other]];
      kcur[s] = pk >> 1;
      ckcur[s] = joint_rows(Jn->type[kin]);
      kids[par[s]].push_back(s);
    }
    // slots are stored leaves first (by height): parents come after children
    for (int s = nsl - 1; s >= 0; --s)
      if (par[s] >= 0) depth[s] = depth[par[s]] + 1;
    std::vector<int> topdown(nsl);
    for (int s = 0; s < nsl; ++s) topdown[s] = s;
    std::stable_sort(topdown.begin(), topdown.end(), [&](int x, int y) { return depth[x] < depth[y]; });
    std::vector<int> nalive(nsl), alive(nsl, 1), sel(nsl, 0), live_child(nsl, -1), raked_child(nsl, 0);
    for (int s = 0; s < nsl; ++s) nalive[s] = (int)kids[s].size();
    int remaining = nsl;
    std::vector<int> chosen;
    while (remaining > 0) {
      const int round0 = (int)c->tc_ops.size();
      c->tc_rounds.push_back(round0);
      for (int s : topdown) {
        if (!alive[s] || nalive[s] != 0) continue;
        TcOp op{};
        op.v = s; op.c = -1; op.kcur = kcur[s]; op.ck = ckcur[s]; op.e = -1; op.ce = 0;
        op.nv = c->tne[s] + ckcur[s];
        c->tc_ops.push_back(op);
      }
      for (int i = c->tc_rounds.back(); i < (int)c->tc_ops.size(); ++i) {
        const int s = c->tc_ops[i].v;
        alive[s] = 0;
        --remaining;
        if (par[s] >= 0) {
          --nalive[par[s]];
          raked_child[par[s]] = 1;
        }
      }
      {  // rakes by clique size: <= 10, <= 16, <= 32, <= 64 rows (TREE_KMAX)
        // operations the kernel runs at once; the 10-row class stays apart
        // (its own kernel, twice the workgroups per CU of the 16-row one)
        // only in rounds large enough to pay for the extra launch
        const int rows[4] = {10, 16, 32, 64};
        const int cap[4] = {1 << 30, 200000, 4096, 1024};
        segment_ops(c->tc_ops, c->tc_rounds, [](const TcOp &o) { return o.nv; }, rows, cap, 4);
      }
      // a compress of v adds the condensed sides of v's other children, and a
      // child raked in this round writes its side in this round: such v wait
      // a round, so that a round's rakes and compresses are independent and
      // share a launch
      chosen.clear();
      for (int s : topdown) {
        if (!alive[s] || par[s] < 0 || nalive[s] != 1 || sel[par[s]] || raked_child[s]) continue;
        int cs = -1;
        for (int k2 : kids[s])
          if (alive[k2]) cs = k2;
        sel[s] = 1;
        chosen.push_back(s);
        live_child[s] = cs;
      }
      for (int s : chosen) {
        const int cs = live_child[s];
        TcOp op{};
        op.v = s; op.c = cs; op.kcur = kcur[s]; op.ck = ckcur[s]; op.e = kcur[cs]; op.ce = ckcur[cs];
        op.nv = c->tne[s] + ckcur[s];
        op.rec = c->crec_size;
        c->crec_size += 55 + 5 * (int64_t)c->tne[cs];
        c->tc_ops.push_back(op);
        // the live child's joint goes last in v's absorbed list
        int e0 = c->tabs_off[s], e1 = c->tabs_off[s + 1];
        for (int e = e0; e < e1; ++e)
          if (abs_joint(c->tabs[e]) == op.e && !(c->tabs[e] & 1)) {
            std::swap(c->tabs[e], c->tabs[e1 - 1]);
            break;
          }
        // merge: c takes v's parent and parent joint
        par[cs] = par[s];
        kcur[cs] = kcur[s];
        ckcur[cs] = ckcur[s];
        for (int &k2 : kids[par[s]])
          if (k2 == s) k2 = cs;
        alive[s] = 0;
        sel[s] = 0;
        --remaining;
      }
      for (int i = round0; i < (int)c->tc_ops.size(); ++i)
        if (c->tc_ops[i].c < 0 && par[c->tc_ops[i].v] >= 0) raked_child[par[c->tc_ops[i].v]] = 0;
      {  // compresses by the larger of v's and c's staged cliques: <= 10, <= 16,
         // <= 32, <= 48 rows, more (team kernels on the global slots)
        const int rows[4] = {10, 16, 32, 48};
        const int cap[4] = {1 << 30, 200000, 2048, 768};
        segment_ops(c->tc_ops, c->tc_rounds,
                    [&](const TcOp &o) { return std::max(o.nv, c->tne[o.c] + std::max(o.ce, o.ck)); }, rows,
                    cap, 4);
      }
    }
    c->tc_rounds.push_back((int)c->tc_ops.size());
    // the paths fork before the third-to-last forward round: the last rounds
    // hold few operations and leave most of the GPU idle (forking before
    // the first round made the path kernels compete with the large rounds;
    // measured on the 4,096-assembly batch: 9.89 ms at round 0, 9.78 ms at
    // round 10 of 13)
    int fork_back = 3;  // MABD_PATH_FORK: forward rounds after the fork
    if (const char *pf = std::getenv("MABD_PATH_FORK")) fork_back = std::max(0, std::atoi(pf));
    c->fork_round = std::max(0, ((int)c->tc_rounds.size() - 1) / TC_NSEG - fork_back);
    // factor slots: K and y with leading dimension absorbed rows + 5, plus
    // the pre-pass scratch of large cliques
    c->foff.clear();
    c->fac_size = 0;
    for (int s = 0; s < nsl; ++s) {
      const int LD = c->tne[s] + 5;
      const int pk = c->tpk[s];
      const int nr0 = c->tne[s] + (pk >= 0 ? joint_rows(Jn->type[c->gj_in[pk >> 1]]) : 0);
      c->foff.push_back(c->fac_size);
      c->fac_size += (int64_t)LD * LD + LD + (nr0 > TREE_KLDS ? 24 * (int64_t)nr0 : 0);
    }
    // what the kernels would otherwise look up per operation
    for (TcOp &op : c->tc_ops) {
      op.av = c->tne[op.v];
      op.ev0 = c->tabs_off[op.v];
      op.ev1 = c->tabs_off[op.v + 1];
      op.fv = c->foff[op.v];
      if (op.c >= 0) {
        op.ac = c->tne[op.c];
        op.ec0 = c->tabs_off[op.c];
        op.ec1 = c->tabs_off[op.c + 1];
        op.fc = c->foff[op.c];
      }
    }
  }
  // ---- path plan: level-0 units (one per path joint) with the clique rows
  // of their bodies, then levels of segments of at most path_T units
  if (c->npath > 0) {
    if (const char *ps = std::getenv("MABD_PATH_SEGMENT")) {  // "T" or "T0,T1"
      int v0 = 0, v1 = 0;
      const int got = std::sscanf(ps, "%d,%d", &v0, &v1);
      if (got >= 1 && v0 >= 2 && v0 <= 64) c->path_T = c->path_T1 = v0;
      if (got == 2 && v1 >= 2 && v1 <= 64) c->path_T1 = v1;
      c->path_T = std::min(c->path_T, PATH_TMAX);
    }
    std::vector<int> pstart;  // first level-0 unit of each path
    for (int p = 0; p < c->npath; ++p) {
      const auto &seq = c->path_j[p];
      pstart.push_back((int)c->pu0.size());
      for (int i = 0; i < (int)seq.size(); ++i) {
        const int k = seq[i];
        PathUnitF u{};
        u.gj = gidx[k];
        u.r = joint_rows(Jn->type[k]);
        const int bb = c->path_bb[p][i], ba = c->path_ba[p][i];
        u.bb = bb >= 0 ? c->in2sol[bb] : -1;
        u.sb = bb >= 0 && Jn->b[k] == bb ? 1 : 0;
        u.ba = ba >= 0 ? c->in2sol[ba] : -1;
        u.sa = ba >= 0 && Jn->b[k] == ba ? 1 : 0;
        c->pu0.push_back(u);
      }
    }
    // levels: each live path's units split evenly into ceil(count / T)
    // segments; the segments' last units are the next level's units
    struct Live { int start, count; };
    std::vector<Live> live;
    std::vector<int32_t> rows_cur;
    for (int p = 0; p < c->npath; ++p) live.push_back({pstart[p], (int)c->path_j[p].size()});
    for (const PathUnitF &u : c->pu0) rows_cur.push_back(u.r);
    PathPlan &P = c->pplan;
    P.seg_off[0] = 0;
    P.unit_off[0] = P.unit_off[1] = 0;
    P.fac_off[0] = 0;
    int lvl = 0;
    while (!live.empty()) {
      if (lvl >= PATH_MAXLEVEL) {
        delete c;
        return fail(nullptr, MABD_ERR_TOPOLOGY, "path component: too many levels");
      }
      std::vector<Live> nxt;
      std::vector<int32_t> rows_next;
      const int seg0 = (int)c->pseg.size();
      const int T = lvl == 0 ? c->path_T : c->path_T1;
      for (const Live &L : live) {
        const int g = (L.count + T - 1) / T;
        int u0 = L.start;
        const int k0 = (int)rows_next.size();
        for (int j = 0; j < g; ++j) {
          PathSeg sg{};
          sg.u0 = u0;
          sg.t = L.count / g + (j < L.count % g ? 1 : 0);
          sg.k = k0 + j;
          sg.flags = (j > 0 ? 1 : 0) | (j == g - 1 ? 2 : 0) | (g == 1 ? 4 : 0);
          c->pseg.push_back(sg);
          rows_next.push_back(rows_cur[u0 + sg.t - 1]);
          u0 += sg.t;
        }
        if (g > 1) nxt.push_back({k0, g});
      }
      const int nseg = (int)c->pseg.size() - seg0;
      P.seg_off[lvl + 1] = (int32_t)c->pseg.size();
      P.fac_off[lvl + 1] = P.fac_off[lvl] + (int64_t)(T - 1) * PATH_FREC * nseg;
      P.unit_off[lvl + 2] = P.unit_off[lvl + 1] + (int64_t)rows_next.size();
      c->prows.insert(c->prows.end(), rows_next.begin(), rows_next.end());
      rows_cur.swap(rows_next);
      live.swap(nxt);
      ++lvl;
    }
    P.nlevel = lvl;
    P.T0 = c->path_T;
  }
  // graph components: bodies after the trees, solved by PCG
  std::vector<int32_t> graph_bodies;
  std::vector<char> gseen(n, 0);
  for (int ci = 0; ci < ncomp; ++ci) {
    if (cls[ci] != CLS_GRAPH) continue;
    // breadth-first order from a body of least degree (Cuthill-McKee): joint
    // neighbours get nearby solver indices, so the PCG gathers stay local
    const auto &bs = cbodies[ci];
    int start = bs[0];
    for (int b : bs)
      if (binc[b].size() < binc[start].size()) start = b;
    std::vector<int> order;
    order.reserve(bs.size());
    order.push_back(start);
    gseen[start] = 1;
    for (size_t head = 0; head < order.size(); ++head) {
      const int b = order[head];
      for (int k : binc[b]) {
        const int o = Jn->a[k] == b ? Jn->b[k] : Jn->a[k];
        if (!dyn(o) || gseen[o]) continue;
        gseen[o] = 1;
        order.push_back(o);
      }
    }
    for (int b : bs)  // the component is connected; kept for safety
      if (!gseen[b]) { gseen[b] = 1; order.push_back(b); }
    for (int b : order) {
      add_body(b);
      graph_bodies.push_back(c->in2sol[b]);
    }
    c->ngraph++;
  }
  c->gb1 = (int)c->sol2in.size();
  c->jmask = gj_graph;
  c->bmask.assign(c->sol2in.size(), 0);
  for (int b : graph_bodies) c->bmask[b] = 1;
  c->nd = (int)c->sol2in.size();
  for (int i = 0; i < n; ++i)
    if (pinned[i]) c->pin_idx.push_back(i);
  c->ns = std::max<int64_t>(((int64_t)c->nd + 63) / 64 * 64, 64);
  // generic joints
  for (int gk = 0; gk < (int)c->gj_in.size(); ++gk) {
    const int k = c->gj_in[gk];
    GJoint g{};
    g.type = Jn->type[k];
    const int a = Jn->a[k], b = Jn->b[k];
    g.sa = dyn(a) ? c->in2sol[a] : -1;
    g.sb = dyn(b) ? c->in2sol[b] : -1;
    const double *pa = Jn->pa + 3 * k, *pb = Jn->pb + 3 * k;
    if (g.sa >= 0) std::memcpy(g.p1a, pa, sizeof g.p1a);
    else world_point(a, pa, g.p1a);
    if (g.sb >= 0) std::memcpy(g.p1b, pb, sizeof g.p1b);
    else world_point(b, pb, g.p1b);
    if (g.type != 0) {
      // rotated-frame joints: the frame dR at rest and the further control
      // points (hinge: P2 on both sides along the axis; universal: b's P2
      // along a2; prismatic: b's P2 along the axis and P3 along the frame's
      // local z); a direction fixed in a's rest frame enters b's rest frame
      // as the same world direction at creation
      double ax[3];
      std::memcpy(ax, Jn->axis + 3 * k, sizeof ax);
      const double nrm = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
      for (double &v : ax) v /= nrm;
      double Ra0[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, Rb0[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
      auto rot0 = [&](int body, double *R) {
        if (body < 0) return;
        const double *q = B->q0 + 12 * body;
        double A[9] = {q[0], q[3], q[6], q[1], q[4], q[7], q[2], q[5], q[8]};
        polar_host(A, R);
      };
      rot0(a, Ra0);
      rot0(b, Rb0);
      double dR[9];
      if (g.type == 2) {
        double a2[3];
        std::memcpy(a2, Jn->axis2 + 3 * k, sizeof a2);
        const double dt = ax[0] * a2[0] + ax[1] * a2[1] + ax[2] * a2[2];
        for (int i = 0; i < 3; ++i) a2[i] -= dt * ax[i];
        const double n2 = std::sqrt(a2[0] * a2[0] + a2[1] * a2[1] + a2[2] * a2[2]);
        for (double &v : a2) v /= n2;
        const double x[3] = {ax[1] * a2[2] - ax[2] * a2[1], ax[2] * a2[0] - ax[0] * a2[2],
                             ax[0] * a2[1] - ax[1] * a2[0]};
        for (int i = 0; i < 3; ++i) {
          dR[i] = x[i];
          dR[3 + i] = ax[i];
          dR[6 + i] = a2[i];
        }
      } else {
        hinge_rod(ax, dR);
      }
      auto in_b = [&](const double *dir_a, double *dir_b) {
        double w[3];
        mat3_vec_h(Ra0, dir_a, w);
        if (b >= 0) mat3t_vec_h(Rb0, w, dir_b);
        else std::memcpy(dir_b, w, sizeof w);
      };
      const double zero[3] = {0.0, 0.0, 0.0};
      double db2[3], db3[3];
      in_b(g.type == 2 ? dR + 6 : ax, db2);
      in_b(g.type == 3 ? dR + 6 : zero, db3);
      const double ell = Jn->cp_len[k];
      double p2a[3], p2b[3], p3b[3];
      for (int i = 0; i < 3; ++i) {
        p2a[i] = pa[i] + ell * ax[i];
        p2b[i] = pb[i] + ell * db2[i];
        p3b[i] = pb[i] + ell * db3[i];
      }
      if (g.sa >= 0) std::memcpy(g.p2a, p2a, sizeof p2a);
      else world_point(a, p2a, g.p2a);
      if (g.sb >= 0) {
        std::memcpy(g.p2b, p2b, sizeof p2b);
        std::memcpy(g.p3b, p3b, sizeof p3b);
      } else {
        world_point(b, p2b, g.p2b);
        world_point(b, p3b, g.p3b);
      }
      if (g.sa >= 0) {
        std::memcpy(g.dR, dR, sizeof dR);
      } else {
        // static frame owner: R_J = dR R_a0^T is constant
        for (int r = 0; r < 3; ++r)
          for (int cc = 0; cc < 3; ++cc)
            g.dR[3 * r + cc] = dR[3 * r] * Ra0[3 * cc] + dR[3 * r + 1] * Ra0[3 * cc + 1] +
                               dR[3 * r + 2] * Ra0[3 * cc + 2];
        g.flags |= GJ_FLAG_STATIC_OWNER;
      }
    }
    c->gj.push_back(g);
  }
  // incidence of generic bodies
  c->inc_off.assign(c->nd + 1, 0);
  {
    std::vector<std::vector<int>> lst(c->nd);
    for (int gk = 0; gk < (int)c->gj.size(); ++gk) {
      if (c->gj[gk].sa >= 0) lst[c->gj[gk].sa].push_back(gk << 1);
      if (c->gj[gk].sb >= 0) lst[c->gj[gk].sb].push_back((gk << 1) | 1);
    }
    for (int i = 0; i < c->nd; ++i) {
      c->inc_off[i + 1] = c->inc_off[i] + (int)lst[i].size();
      for (int e : lst[i]) c->inc.push_back(e);
    }
  }
  // shapes
  std::vector<double> shape;
  std::vector<int32_t> shp(c->nd);
  {
    std::map<std::tuple<double, double, double, double, double, double>, int> dedup;
    for (int s = 0; s < c->nd; ++s) {
      const int i = c->sol2in[s];
      const double *d = B->dims + 3 * i;
      const double nu = opt.material == 1 ? B->poisson[i] : 0.0;
      auto key = std::make_tuple(d[0], d[1], d[2], B->density[i], B->k_orth[i], nu);
      auto it = dedup.find(key);
      if (it == dedup.end()) {
        it = dedup.emplace(key, (int)dedup.size()).first;
        const double V = d[0] * d[1] * d[2], mass = B->density[i] * V;
        double mu, lam;
        if (opt.material == 1) {
          mu = B->k_orth[i] / (2.0 * (1.0 + nu));
          lam = B->k_orth[i] * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        } else {
          mu = 4.0 * B->k_orth[i];  // Eq. EA linearised at rest
          lam = 0.0;
        }
        const double rec[SHAPE_STRIDE] = {mass * d[0] * d[0] / 12.0, mass * d[1] * d[1] / 12.0,
                                          mass * d[2] * d[2] / 12.0, mass, V, mu, lam, 0.0};
        shape.insert(shape.end(), rec, rec + SHAPE_STRIDE);
      }
      shp[s] = it->second;
    }
    c->nshape = (int)dedup.size();
  }

  // ------------------------------------------------------------ device
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  if (opt.stream) {
    c->stream = (hipStream_t)opt.stream;
  } else {
    chk(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  const int64_t ns = c->ns;
  for (int pb = 0; pb < 2; ++pb) {
    chk(dalloc(c, &c->d_q[pb], 12 * ns));
    chk(dalloc(c, &c->d_qd[pb], 12 * ns));
  }
  {
    std::vector<double> hq(12 * ns, 0.0), hqd(12 * ns, 0.0);
    for (int s = 0; s < c->nd; ++s)
      for (int cc = 0; cc < 12; ++cc) {
        hq[cc * ns + s] = c->q0_in[12 * (size_t)c->sol2in[s] + cc];
        hqd[cc * ns + s] = c->qd0_in[12 * (size_t)c->sol2in[s] + cc];
      }
    if (e == hipSuccess) chk(hipMemcpy(c->d_q[0], hq.data(), hq.size() * 8, hipMemcpyHostToDevice));
    if (e == hipSuccess) chk(hipMemcpy(c->d_qd[0], hqd.data(), hqd.size() * 8, hipMemcpyHostToDevice));
  }
  if (e == hipSuccess) chk(upload(c, &c->d_shp, shp));
  if (e == hipSuccess) chk(upload(c, &c->d_shape, shape));
  if (e == hipSuccess) chk(dalloc(c, &c->d_hinv, (size_t)HINV_STRIDE * c->nshape));
  if (e == hipSuccess) chk(upload(c, &c->d_chains, c->chains));
  if (e == hipSuccess) chk(upload(c, &c->d_tiles, c->tiles));
  const int64_t nrs = std::max<int64_t>(c->nchain_rows, 1);
  {
    std::vector<double> spl(3 * nrs, 0.0), spr(3 * nrs, 0.0);
    for (int r = 0; r < c->nchain_rows; ++r)
      for (int i = 0; i < 3; ++i) {
        spl[i * nrs + r] = pl[3 * r + i];
        spr[i * nrs + r] = pr[3 * r + i];
      }
    if (e == hipSuccess) chk(upload(c, &c->d_pl, spl));
    if (e == hipSuccess) chk(upload(c, &c->d_pr, spr));
    if (e == hipSuccess) chk(upload(c, &c->d_flag, cflag));
  }
  if (e == hipSuccess) chk(dalloc(c, &c->d_tilerec, (size_t)TILE_REC * c->tiles.size()));
  if (e == hipSuccess) chk(upload(c, &c->d_groups, c->groups));
  if (e == hipSuccess) chk(dalloc(c, &c->d_grouprec, (size_t)TILE_REC * c->groups.size()));
  if (e == hipSuccess) chk(dalloc(c, &c->d_gfac, (size_t)PACK_CF * CHAIN_THREADS * c->groups.size()));
  if (e == hipSuccess) chk(dalloc(c, &c->d_xtop, (size_t)3 * c->ntop));
  if (e == hipSuccess) chk(dalloc(c, &c->d_gcount, std::max<size_t>(c->chains.size(), 1)));
  {
    const size_t ngrp = (c->tiles.size() + 3) / 4;
    if (e == hipSuccess) chk(dalloc(c, &c->d_psv, (size_t)PACK_SV * 64 * ngrp));
    if (e == hipSuccess) chk(dalloc(c, &c->d_pcf, (size_t)PACK_CF * 64 * ngrp));
  }
  if (e == hipSuccess) chk(hipMemset(c->d_gcount, 0, std::max<size_t>(c->chains.size(), 1) * sizeof(int)));
  if (e == hipSuccess) chk(dalloc(c, &c->d_grow, (size_t)GROW_REC * c->ntop));
  if (e == hipSuccess) chk(dalloc(c, &c->d_xg, (size_t)3 * c->ngrows));
  if (e == hipSuccess) chk(dalloc(c, &c->d_clam, (size_t)3 * nrs));
  if (opt.precision == 1 && !c->chains.empty()) {
    if (e == hipSuccess) chk(dalloc(c, &c->d_dq, (size_t)12 * ns));
    if (e == hipSuccess) chk(dalloc(c, &c->d_rp, (size_t)12 * ns));
    if (e == hipSuccess) chk(dalloc(c, &c->d_rd, (size_t)3 * nrs));
    if (e == hipSuccess) chk(dalloc(c, &c->d_part, (size_t)IR_PART * c->tiles.size()));
    if (e == hipSuccess) chk(dalloc(c, &c->d_ir, 8));
    if (e == hipSuccess) chk(hipMemset(c->d_ir, 0, 8 * sizeof(double)));
    if (e == hipSuccess) chk(hipHostMalloc((void **)&c->h_ir, 8 * sizeof(double)));
  }
  if (e == hipSuccess) chk(upload(c, &c->d_gj, c->gj));
  if (e == hipSuccess) {
    std::vector<uint8_t> jr(c->gj.size());
    for (size_t k = 0; k < c->gj.size(); ++k) jr[k] = (uint8_t)joint_rows(c->gj[k].type);
    chk(upload(c, &c->d_jrows, jr));
  }
  const size_t mg = c->gj.size();
  if (e == hipSuccess) chk(dalloc(c, &c->d_gl, GL_STRIDE * mg));
  if (e == hipSuccess) chk(dalloc(c, &c->d_gt, GT_STRIDE * mg));
  if (e == hipSuccess) chk(dalloc(c, &c->d_glam, 5 * mg));
  if (e == hipSuccess) chk(dalloc(c, &c->d_Rg, 9 * ns));
  if (e == hipSuccess) chk(dalloc(c, &c->d_ug, 12 * ns));
  if (e == hipSuccess) chk(upload(c, &c->d_comp_lvl, c->comp_lvl));
  if (e == hipSuccess) chk(upload(c, &c->d_lvl_off, c->lvl_off));
  if (e == hipSuccess) chk(upload(c, &c->d_tbody, c->tbody));
  if (e == hipSuccess) chk(upload(c, &c->d_tpk, c->tpk));
  if (e == hipSuccess) chk(upload(c, &c->d_tabs_off, c->tabs_off));
  if (e == hipSuccess) chk(upload(c, &c->d_tabs, c->tabs));
  if (e == hipSuccess) chk(upload(c, &c->d_tne, c->tne));
  if (e == hipSuccess) chk(upload(c, &c->d_foff, c->foff));
  if (e == hipSuccess) chk(dalloc(c, &c->d_fac, (size_t)std::max<int64_t>(c->fac_size, 1)));
  if (e == hipSuccess) chk(upload(c, &c->d_tc_ops, c->tc_ops));
  if (e == hipSuccess) chk(dalloc(c, &c->d_crec, (size_t)std::max<int64_t>(c->crec_size, 1)));
  if (c->npath > 0) {
    PathPlan &P = c->pplan;
    const int64_t nu = std::max<int64_t>(P.unit_off[P.nlevel + 1], 1);
    PathUnitF *du0 = nullptr;
    PathSeg *dseg = nullptr;
    int32_t *drows = nullptr;
    if (e == hipSuccess) chk(upload(c, &du0, c->pu0));
    if (e == hipSuccess) chk(upload(c, &dseg, c->pseg));
    if (e == hipSuccess) {
      if (c->prows.empty()) c->prows.push_back(0);
      chk(upload(c, &drows, c->prows));
    }
    if (e == hipSuccess) chk(dalloc(c, &P.unit, (size_t)(PATH_UREC * nu)));
    if (e == hipSuccess) chk(dalloc(c, &P.lam, (size_t)(5 * nu)));
    if (e == hipSuccess) chk(dalloc(c, &P.fac, (size_t)std::max<int64_t>(P.fac_off[P.nlevel], 1)));
    P.uf = du0;
    P.seg = dseg;
    P.rows = drows;
  }
  if (c->nloop > 0) {
    if (e == hipSuccess) chk(upload(c, &c->d_jloop, c->jloop));
    if (e == hipSuccess) chk(upload(c, &c->d_loff, c->loff));
    if (e == hipSuccess) chk(upload(c, &c->d_lrow, c->lrow));
    if (e == hipSuccess) chk(dalloc(c, &c->d_lamD, c->lrow.size()));
    if (e == hipSuccess) chk(dalloc(c, &c->d_uloop, 12 * (size_t)ns));
    if (e == hipSuccess) chk(hipMemset(c->d_uloop, 0, 12 * (size_t)ns * sizeof(double)));
    if (e == hipSuccess) chk(dalloc(c, &c->d_wcol, (size_t)c->loop_maxr * 5 * mg));
  }
  if (e == hipSuccess) chk(upload(c, &c->d_inc_off, c->inc_off));
  if (e == hipSuccess) chk(upload(c, &c->d_inc, c->inc));
  if (e == hipSuccess) chk(upload(c, &c->d_sol2in, c->sol2in));
  if (e == hipSuccess) chk(upload(c, &c->d_pin_idx, c->pin_idx));
  {
    std::vector<double> pq;
    for (int i : c->pin_idx) pq.insert(pq.end(), c->q0_in.begin() + 12 * (size_t)i, c->q0_in.begin() + 12 * (size_t)i + 12);
    if (e == hipSuccess) chk(upload(c, &c->d_pin_q0, pq));
  }
  if (e == hipSuccess) chk(dalloc(c, &c->d_tmp, (size_t)24 * std::max(n, 1)));
  if (c->ngraph > 0) {
    if (e == hipSuccess) chk(upload(c, &c->d_jmask, c->jmask));
    if (e == hipSuccess) chk(upload(c, &c->d_bmask, c->bmask));
    if (e == hipSuccess) chk(dalloc(c, &c->d_pr_, 5 * mg));
    if (e == hipSuccess) chk(dalloc(c, &c->d_pp, 5 * mg));
    if (e == hipSuccess) chk(dalloc(c, &c->d_pz, 5 * mg));
    if (e == hipSuccess) chk(dalloc(c, &c->d_psp, 5 * mg));
    if (e == hipSuccess) chk(dalloc(c, &c->d_pbv, 5 * mg));
    if (e == hipSuccess) chk(dalloc(c, &c->d_dinv, 25 * mg));
    if (e == hipSuccess) chk(dalloc(c, &c->d_zb, 12 * ns));
    if (e == hipSuccess) {
      c->pcg_blocks = std::min(pcg_max_blocks(), (int)std::max<size_t>((mg + 255) / 256, 1));
      if (c->pcg_blocks <= 0) e = hipErrorInvalidConfiguration;
    }
    // compact ball-joint operator
    bool allball = true;
    for (size_t k = 0; k < c->gj.size(); ++k)
      if (c->jmask[k] && c->gj[k].type != 0) allball = false;
    if (allball && e == hipSuccess) {
      std::vector<int32_t> bpos(c->sol2in.size(), -1), bid, jid, jba, jbb;
      for (int b = c->gb0; b < c->gb1; ++b)
        if (c->bmask[b]) { bpos[b] = (int)bid.size(); bid.push_back(b); }
      for (size_t k = 0; k < c->gj.size(); ++k)
        if (c->jmask[k]) jid.push_back((int)k);
      // joints in the order of their first dynamic body (locality of gathers)
      auto key = [&](int k) {
        const GJoint &g = c->gj[k];
        const int a = g.sa >= 0 ? bpos[g.sa] : INT32_MAX, b = g.sb >= 0 ? bpos[g.sb] : INT32_MAX;
        return std::make_pair(std::min(a, b), std::max(a, b));
      };
      std::stable_sort(jid.begin(), jid.end(), [&](int x, int y) { return key(x) < key(y); });
      const int nj = (int)jid.size(), nbd = (int)bid.size();
      std::vector<double> jp(8 * (size_t)std::max(nj, 1), 0.0);
      std::vector<int32_t> boff(nbd + 1, 0), binc;
      jba.resize(nj);
      jbb.resize(nj);
      for (int j = 0; j < nj; ++j) {
        const GJoint &g = c->gj[jid[j]];
        jba[j] = g.sa >= 0 ? bpos[g.sa] : -1;
        jbb[j] = g.sb >= 0 ? bpos[g.sb] : -1;
        for (int q = 0; q < 3; ++q) {
          jp[8 * (size_t)j + q] = g.p1a[q];
          jp[8 * (size_t)j + 3 + q] = g.p1b[q];
        }
        if (jba[j] >= 0) boff[jba[j] + 1]++;
        if (jbb[j] >= 0) boff[jbb[j] + 1]++;
      }
      for (int i = 0; i < nbd; ++i) boff[i + 1] += boff[i];
      binc.assign(std::max(boff[nbd], 1), 0);
      {
        std::vector<int32_t> fill(boff.begin(), boff.end() - 1);
        for (int j = 0; j < nj; ++j) {
          if (jba[j] >= 0) binc[fill[jba[j]]++] = j << 1;
          if (jbb[j] >= 0) binc[fill[jbb[j]]++] = (j << 1) | 1;
        }
      }
      c->pcg_ball = true;
      c->pb_nj = nj;
      c->pb_nbd = nbd;
      chk(upload(c, &c->d_pb_jid, jid));
      if (e == hipSuccess) chk(upload(c, &c->d_pb_jba, jba));
      if (e == hipSuccess) chk(upload(c, &c->d_pb_jbb, jbb));
      if (e == hipSuccess) chk(upload(c, &c->d_pb_bid, bid));
      if (e == hipSuccess) chk(upload(c, &c->d_pb_boff, boff));
      if (e == hipSuccess) chk(upload(c, &c->d_pb_binc, binc));
      if (e == hipSuccess) chk(upload(c, &c->d_pb_jp, jp));
      if (e == hipSuccess) chk(dalloc(c, &c->d_pb_vec, (size_t)7 * 3 * std::max(nj, 1)));
      if (e == hipSuccess) chk(dalloc(c, &c->d_pb_dinv, (size_t)6 * std::max(nj, 1)));
      if (e == hipSuccess) chk(dalloc(c, &c->d_pb_zw, (size_t)16 * std::max(nbd, 1)));
      if (e == hipSuccess) chk(dalloc(c, &c->d_pb_sc, 8));
      if (e == hipSuccess) chk(dalloc(c, &c->d_pb_si, 8));
      if (e == hipSuccess) chk(hipHostMalloc((void **)&c->h_pb_si, 8 * sizeof(int32_t)));
      c->pb_blocks = std::max(1, (nj + 255) / 256);  // joint blocks: one partial slot set each
      c->pcg_blocks = std::max(c->pcg_blocks, c->pb_blocks);
    }
    if (e == hipSuccess) chk(dalloc(c, &c->d_partial, 4 * (size_t)std::max(c->pcg_blocks, 1)));
    if (e == hipSuccess) chk(dalloc(c, &c->d_pcg_res, 2));
    if (e == hipSuccess) chk(dalloc(c, &c->d_pcg_it, 2));
    if (e == hipSuccess) chk(hipHostMalloc((void **)&c->h_pcg, 4 * sizeof(double)));
  }
  if (e == hipSuccess && mg) chk(hipMemset(c->d_glam, 0, 5 * mg * sizeof(double)));
  if (e == hipSuccess) chk(dalloc(c, &c->d_status, 4));
  if (e == hipSuccess) chk(hipHostMalloc((void **)&c->h_status, 4 * sizeof(uint32_t)));
  if (e == hipSuccess) chk(hipEventCreateWithFlags(&c->pend_ev, hipEventDisableTiming));
  // (a few short paths beside a large tree are not worth the fork's events)
  if (e == hipSuccess && c->pu0.size() >= 16384 && !c->tbody.empty()) {
    chk(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    if (e == hipSuccess) chk(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    if (e == hipSuccess) chk(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  }
  {
    // the fixed scratch of mabd_residual_noalloc on this (current) device
    int dev = 0;
    if (e == hipSuccess) chk(hipGetDevice(&dev));
    if (e == hipSuccess) chk(resid_scratch(dev, &c->d_rscratch));
  }
  if (e == hipSuccess) chk(dalloc(c, &c->d_diag, DIAG_VALUES));
  if (e == hipSuccess) chk(hipHostMalloc((void **)&c->h_diag, DIAG_VALUES * sizeof(double)));
  // precision form 1 on the generic components: one Newton iteration, no
  // loop or network component (those stay FP64)
  c->gen_ir = opt.precision == 1 && opt.newton_iters == 1 && c->gb1 > c->gb0 && c->ngraph == 0 &&
              c->nloop == 0;
  if (c->gen_ir) {
    const size_t mgi = std::max<size_t>(c->gj.size(), 1);
    if (e == hipSuccess) chk(dalloc(c, &c->d_uc, (size_t)12 * ns));
    if (e == hipSuccess) chk(dalloc(c, &c->d_cc, 5 * mgi));
    if (e == hipSuccess) chk(dalloc(c, &c->d_dlam, 5 * mgi));
    if (e == hipSuccess)
      chk(dalloc(c, &c->d_irpart, (size_t)DIAG_PART * (diag_body_blocks(c->gb1 - c->gb0) +
                                                      diag_body_blocks((int)c->gj.size()))));
    if (e == hipSuccess) chk(dalloc(c, &c->d_irout, 5));
    if (e == hipSuccess) chk(hipHostMalloc((void **)&c->h_irout, 6 * sizeof(double)));
  }
  if (opt.diagnostics & 1) {
    // sized here, while the tiles are the smallest (most numerous) form
    if (e == hipSuccess) chk(dalloc(c, &c->d_dpart, (size_t)DIAG_PART * diag_nblk(c)));
    if (opt.newton_iters > 1 && c->gb1 > c->gb0) {
      if (e == hipSuccess) chk(dalloc(c, &c->d_qit, (size_t)12 * ns));
      if (e == hipSuccess) chk(dalloc(c, &c->d_dqit, (size_t)12 * ns));
    }
  }
  // after every buffer is sized for the smallest tiles
  // "64p" (packed), 64, 128 or 256: fixed by the environment, no autotuning
  if (const char *tt = std::getenv("MABD_CHAIN_TILE_THREADS")) {
    const std::string v(tt);
    const bool pack = v == "64p";
    const int n = pack ? 64 : std::atoi(tt);
    if (pack || v == "64" || v == "128" || v == "256") {
      c->tuned = true;
      if (e == hipSuccess) chk(build_tiles(c, n, pack));
    }
  }
  if (e != hipSuccess) {
    mabd_status st = (e == hipErrorOutOfMemory) ? MABD_ERR_OOM : MABD_ERR_DEVICE;
    std::string msg = std::string("device setup failed: ") + hipGetErrorString(e);
    mabd_destroy(c);
    return fail(nullptr, st, msg);
  }
  c->stats.n_chain = (int)c->chains.size();
  c->stats.n_tree = c->ntree;
  c->stats.n_path = c->npath;
  c->stats.path_levels = c->npath > 0 ? c->pplan.nlevel : 0;
  c->stats.n_graph = c->ngraph;
  c->stats.n_loop = c->nloop;
  c->stats.n_dyn = c->nd;
  if (e == hipSuccess && !c->tuned && opt.autotune && (tune_chain(c) || tune_tree(c))) {
    int tt, pk, split, order;
    if (tune_cache_read(c, tt, pk, split, order)) {
      if (!c->chains.empty()) e = build_tiles(c, tt, pk != 0);
      c->tree_split = split;
      c->tree_order = order;
      c->tuned = true;
      c->tune_source = 2;
      if (e != hipSuccess) {
        mabd_destroy(c);
        return fail(nullptr, MABD_ERR_DEVICE, std::string("device setup failed: ") + hipGetErrorString(e));
      }
    }
  }
  c->stats.tile_threads = c->tile_threads;
  c->stats.tile_packed = c->tile_pack ? 1 : 0;
  c->stats.tree_split = c->tree_split;
  c->stats.tree_order = c->tree_order;
  c->stats.tune_source = c->tune_source;
  c->stats.tree_rounds = ((int)c->tc_rounds.size() - 1) / TC_NSEG;
  c->stats.rho_p = c->stats.rho_d = c->stats.kkt = -1.0;
  *out = c;
  return MABD_OK;
}


}  // extern "C"

namespace {
// arguments of the ball-network operator and PCG
PcgBallArgs make_ball_args(mabd_ctx *c, double tol, int max_iters, int warm) {
  PcgBallArgs pb{};
  pb.nj = c->pb_nj;
  pb.nbd = c->pb_nbd;
  pb.jid = c->d_pb_jid;
  pb.jba = c->d_pb_jba;
  pb.jbb = c->d_pb_jbb;
  pb.jp = c->d_pb_jp;
  pb.bid = c->d_pb_bid;
  pb.binc_off = c->d_pb_boff;
  pb.binc = c->d_pb_binc;
  pb.gl = c->d_gl;
  pb.Rg = c->d_Rg;
  pb.ug = c->d_ug;
  pb.ns = c->ns;
  pb.shp = c->d_shp;
  pb.hinv = c->d_hinv;
  pb.glam = c->d_glam;
  const size_t v3 = (size_t)3 * std::max(c->pb_nj, 1);
  pb.x = c->d_pb_vec;
  pb.r = c->d_pb_vec + v3;
  pb.z = c->d_pb_vec + 2 * v3;
  pb.p0 = c->d_pb_vec + 3 * v3;
  pb.p1 = c->d_pb_vec + 4 * v3;
  pb.sp = c->d_pb_vec + 5 * v3;
  pb.bv = c->d_pb_vec + 6 * v3;
  pb.dinv = c->d_pb_dinv;
  pb.zw = c->d_pb_zw;
  pb.partial = c->d_partial;
  pb.nblk = c->pb_blocks;
  pb.sc = c->d_pb_sc;
  pb.si = c->d_pb_si;
  pb.tol = tol;
  pb.max_iters = max_iters;
  pb.warm = warm;
  pb.iters_out = c->d_pcg_it;
  pb.res_out = c->d_pcg_res;
  pb.status = c->d_status;
  pb.step = 0;
  return pb;
}
}  // namespace

namespace {
void drop_graphs(mabd_ctx *c);

// ------------------------------------------------------ learned warm start
hipError_t gnn_alloc(mabd_ctx *c) {
  if (c->gnn_ready) return hipSuccess;
  const size_t nj = (size_t)std::max(c->pb_nj, 1), nbd = (size_t)std::max(c->pb_nbd, 1);
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  GnnBufs &g = c->gb;
  chk(dalloc(c, &g.x0, GNN_FIN * nj));
  for (int l = 0; l < GNN_L; ++l) chk(dalloc(c, &g.X[l], 2 * GNN_W * nj));
  for (int l = 0; l <= GNN_L; ++l) chk(dalloc(c, &g.H[l], GNN_W * nj));
  chk(dalloc(c, &g.y, 3 * nj));
  chk(dalloc(c, &g.m, GNN_W * nbd));
  chk(dalloc(c, &g.dX, 2 * GNN_W * nj));
  chk(dalloc(c, &g.dZ, GNN_W * nj));
  chk(dalloc(c, &g.dY, 3 * nj));
  chk(dalloc(c, &g.params, (size_t)GNN_NPARAM));
  chk(dalloc(c, &g.grad, (size_t)GNN_NPARAM));
  chk(dalloc(c, &g.adam_m, (size_t)GNN_NPARAM));
  chk(dalloc(c, &g.adam_v, (size_t)GNN_NPARAM));
  chk(dalloc(c, &g.wpart, (size_t)gnn_wgrad_blocks((int)nj) * (2 * GNN_W + 1) * GNN_W));
  chk(dalloc(c, &g.lb, 3 * nj));
  chk(dalloc(c, &g.rb, 3 * nj));
  chk(dalloc(c, &g.red, 4 * ((nj + 255) / 256)));
  chk(dalloc(c, &g.sc, 8));
  if (e == hipSuccess && !c->h_gsc) e = hipHostMalloc((void **)&c->h_gsc, 4 * sizeof(double));
  return e;
}

hipError_t gnn_set_params(mabd_ctx *c, const float *P) {
  hipError_t e = hipMemcpy(c->gb.params, P, GNN_NPARAM * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->gb.adam_m, 0, GNN_NPARAM * sizeof(float));
  if (e == hipSuccess) e = hipMemset(c->gb.adam_v, 0, GNN_NPARAM * sizeof(float));
  c->gnn_t = 0;
  if (e == hipSuccess) c->gnn_ready = true;
  return e;
}

// Glorot-uniform weights from a splitmix64 stream, zero biases; the decoder is
// scaled by 0.1 so that an untrained network starts near zero
void gnn_init_params(std::vector<float> &P, uint64_t seed) {
  P.assign(GNN_NPARAM, 0.0f);
  uint64_t st = seed;
  auto uni = [&]() {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  auto glorot = [&](int off, int fin, int fout, double gain) {
    const double a = gain * std::sqrt(6.0 / (fin + fout));
    for (int i = 0; i < fin * fout; ++i) P[off + i] = (float)((2.0 * uni() - 1.0) * a);
  };
  glorot(GNN_P_WE, GNN_FIN, GNN_W, 1.0);
  for (int l = 0; l < GNN_L; ++l) glorot(GNN_P_L0 + l * GNN_P_LSTRIDE, 2 * GNN_W, GNN_W, 1.0);
  glorot(GNN_P_WD, GNN_W, 3, 0.1);
}

// The dual system of the current state (per-body solve, joint rows, PCG
// diagonal blocks and right-hand side) without advancing the state.
hipError_t gnn_prepare(mabd_ctx *c, double h, PcgBallArgs &pb) {
  hipStream_t s = c->stream;
  if (h != c->h_last) {
    launch_prefactor(c->d_shape, c->nshape, h, c->d_hinv, s);
    c->h_last = h;
    drop_graphs(c);
  }
  launch_reset_status(c->d_status, s);
  launch_begin_step(c->d_status, s);
  const int a = c->cur;
  launch_gbody(c->gb0, c->gb1, c->d_q[a], c->d_q[a], c->d_qd[a], c->ns, c->d_shp, c->d_hinv, c->d_shape,
               c->opt.gravity, h, c->d_Rg, c->d_ug, c->d_status, 0, c->wr_on ? c->d_wr : nullptr,
               nullptr, 0, nullptr, nullptr, nullptr, 0, nullptr, s);  // network bodies have joints: the polar solve
  launch_gjoint((int)c->gj.size(), c->d_gj, c->d_q[a], c->d_Rg, c->ns, c->opt.hinge_grad, c->d_gl, s);
  pb = make_ball_args(c, c->opt.kkt_tol, c->opt.max_iters, 0);
  launch_pb_setup(pb, s);
  return hipGetLastError();
}

mabd_status gnn_check(mabd_ctx *c, bool need_ready) {
  if (!c) return MABD_ERR_INVALID_ARG;
  const mabd_status rs = resolve(c);  // these calls clear the status word
  if (rs != MABD_OK) return rs;
  c->resid_ok = false;  // and overwrite the step's rows and local solves
  if (!c->pcg_ball || c->pb_nj == 0)
    return fail(c, MABD_ERR_INVALID_ARG, "the learned warm start needs a ball-joint network component");
  if (need_ready && !c->gnn_ready)
    return fail(c, MABD_ERR_INVALID_ARG, "no network weights: call mabd_gnn_init or mabd_gnn_load");
  return MABD_OK;
}

mabd_status gnn_finish(mabd_ctx *c, const char *what) {
  hipError_t e = hipMemcpyAsync(c->h_status, c->d_status, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  if (c->h_status[0] & FLAG_NONFINITE) return fail(c, MABD_ERR_NONFINITE, std::string(what) + ": non-finite state");
  if (c->h_status[0] & FLAG_SINGULAR) return fail(c, MABD_ERR_SINGULAR, std::string(what) + ": singular block");
  return MABD_OK;
}
}  // namespace


namespace {
// Ball-joint PCG: setup and start on the device, then chunks of iterations
// with a read of the flags after each chunk (chunk lengths double from 8 to
// 256, all even, so every chunk starts on an even iteration).  When the
// recursive residual passes, the true residual decides: done, or a restart
// from it (at most four).
hipError_t run_pcg_ball(mabd_ctx *c, const PcgBallArgs &pb, hipStream_t s) {
  enum { SI_DONE = 0, SI_CONV = 1, SI_ITERS = 2, SI_FINAL = 3, SI_BAD = 4 };
  launch_pb_setup(pb, s);
  c->stats.warm_accepted = 0;
  if (c->opt.warm_start == 2 && c->gnn_ready) {
    // learned correction of the base start (previous multipliers, or zero),
    // kept only if it lowers the dual energy, i.e. the S-norm error
    const int prev = c->warm_valid ? 1 : 0;
    launch_gnn_forward(pb, c->gb, prev, s);
    launch_gnn_loss(pb, c->gb, s);
    hipError_t e = hipMemcpyAsync(c->h_gsc, c->gb.sc + 3, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (c->h_gsc[0] < 0.0) {
      c->stats.warm_accepted = 1;
      launch_gnn_add_base(pb, c->gb, s);
      launch_pb_residual(pb, 1, 0, s);
    } else {
      PcgBallArgs base = pb;
      base.warm = prev;
      launch_pb_setup(base, s);  // x = the base start again
      launch_pb_residual(base, prev, 0, s);
    }
  } else {
    launch_pb_residual(pb, pb.warm, 0, s);
  }
  int chunk = 8, restarts = 0;
  bool first = true;
  hipError_t e = hipSuccess;
  for (;;) {
    e = hipMemcpyAsync(c->h_pb_si, pb.si, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    const int32_t *si = c->h_pb_si;
    if (si[SI_FINAL] || si[SI_BAD]) break;
    if (si[SI_DONE]) {
      if (!si[SI_CONV] || restarts >= 4) break;  // iteration cap, or no restarts left
      ++restarts;
      launch_pb_residual(pb, 1, 1, s);  // true residual: ends the solve or restarts it
      first = true;
      continue;
    }
    launch_pb_iters(pb, chunk, first ? 1 : 0, s);
    first = false;
    chunk = std::min(chunk * 2, 256);
  }
  launch_pb_finish(pb, s);
  return hipGetLastError();
}

// Arguments of the chain kernels for a step reading state buffer a and
// writing buffer b.
ChainArgs chain_args(mabd_ctx *c, double h, int a, int b) {
  const double *g = c->opt.gravity;
  ChainArgs ca{};
  ca.chains = c->d_chains;
  ca.tiles = c->d_tiles;
  ca.ntiles = (int)c->tiles.size();
  ca.q = c->d_q[a];
  ca.qd = c->d_qd[a];
  ca.q_out = c->d_q[b];
  ca.qd_out = c->d_qd[b];
  ca.ns = c->ns;
  ca.shp = c->d_shp;
  ca.hinv = c->d_hinv;
  ca.shape = c->d_shape;
  ca.pl = c->d_pl;
  ca.pr = c->d_pr;
  ca.flag = c->d_flag;
  ca.nrs = std::max(c->nchain_rows, 1);
  ca.g[0] = g[0]; ca.g[1] = g[1]; ca.g[2] = g[2];
  ca.h = h;
  ca.tilerec = c->d_tilerec;
  ca.xg = c->d_xg;
  ca.lam = c->d_clam;
  ca.status = c->d_status;
  ca.step = 0;
  ca.dq = c->d_dq;
  ca.rp = c->d_rp;
  ca.rd = c->d_rd;
  ca.part = c->d_part;
  ca.ir = c->d_ir;
  ca.wr = c->wr_on ? c->d_wr : nullptr;
  ca.psv = c->d_psv;
  ca.pcf = c->d_pcf;
  ca.diag = 0;
  return ca;
}

// Residual kernels of one finished Newton iteration into `part` (diag_nblk
// records) and their reduction into out[0..4] (diag_reduce_kernel).  The
// step read state buffer a and wrote buffer b.  Chains (fused path, one
// iteration) recompute their forces from buffer a and take their increment
// as h times the new velocity; generic bodies take the iterate q_it and the
// increment dq_scale * dqv.
void issue_residual(mabd_ctx *c, double h, int a, int b, const double *q_it, const double *dqv,
                    double dq_scale, double *part, double *out) {
  hipStream_t s = c->stream;
  int64_t off = 0;
  if (!c->chains.empty()) {
    ChainArgs ca = chain_args(c, h, a, b);
    ca.diag = 1;
    ca.part = part;
    launch_chain_resid(ca, (int)c->tiles.size(), c->tile_threads, s);
  }
  off += (int64_t)c->tiles.size();
  launch_gdiag_body(c->gb0, c->gb1, q_it, c->d_q[a], c->d_qd[a], dqv, dq_scale, c->ns, c->d_shp,
                    c->d_hinv, c->d_shape, c->opt.gravity, h, c->d_Rg, c->d_inc_off, c->d_inc, c->d_gj,
                    c->d_gl, c->d_glam, c->wr_on ? c->d_wr : nullptr, c->d_status,
                    part + DIAG_PART * off, c->opt.body_solve, nullptr, s);
  off += diag_body_blocks(c->gb1 - c->gb0);
  launch_gdiag_joint((int)c->gj.size(), c->d_gj, c->d_gl, c->d_Rg, c->d_ug, dqv, dq_scale, c->d_q[b],
                     c->ns, c->d_status, part + DIAG_PART * off, nullptr, s);
  off += diag_body_blocks((int)c->gj.size());
  launch_diag_reduce(part, (int)off, out, c->d_status, s);
}

// Precision form 1 on the generic components (trees): after the FP32 solve
// of the step, the FP64 KKT residual of the generic bodies and joints (read
// by the host) decides: converged, stalled at the rounding floor (a sweep
// that no longer halves it; accepted within 10 kkt_tol), or a correction
// sweep: the same tree solve with Hbar^{-1} R^T r_p in place of u and r_d
// in place of C, whose increment and multipliers are added to the step's.
// Host-controlled: each check waits for the stream.
hipError_t generic_refine(mabd_ctx *c, double h, int a, int b, const TreeArgs &ta) {
  hipStream_t s = c->stream;
  const int mg = (int)c->gj.size();
  const double tol = c->opt.kkt_tol;
  const int nsw = c->opt.ir_max_sweeps;
  c->gir_sweeps = 0;
  c->gir_stalled = 0;
  c->gir_rho_p = c->gir_rho_d = c->gir_kkt = -1.0;
  double prev = 0.0;
  for (int sw = 0;; ++sw) {
    const bool last = sw == nsw;
    double *uc = last ? nullptr : c->d_uc, *cc = last ? nullptr : c->d_cc;
    launch_gdiag_body(c->gb0, c->gb1, c->d_q[a], c->d_q[a], c->d_qd[a], c->d_qd[b], h, c->ns, c->d_shp,
                      c->d_hinv, c->d_shape, c->opt.gravity, h, c->d_Rg, c->d_inc_off, c->d_inc, c->d_gj,
                      c->d_gl, c->d_glam, c->wr_on ? c->d_wr : nullptr, c->d_status, c->d_irpart,
                      c->opt.body_solve, uc, s);
    const int off = diag_body_blocks(c->gb1 - c->gb0);
    launch_gdiag_joint(mg, c->d_gj, c->d_gl, c->d_Rg, c->d_ug, c->d_qd[b], h, c->d_q[b], c->ns, c->d_status,
                       c->d_irpart + DIAG_PART * (int64_t)off, cc, s);
    launch_diag_reduce(c->d_irpart, off + diag_body_blocks(mg), c->d_irout, c->d_status, s);
    hipError_t e = hipMemcpyAsync(c->h_irout, c->d_irout, 5 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->h_irout + 5, c->d_status, 2 * sizeof(uint32_t),
                                            hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    uint32_t st[2];
    std::memcpy(st, c->h_irout + 5, sizeof st);
    if (st[0] != 0u) return hipSuccess;  // an earlier failure of this step: nothing to refine
    const double kkt = c->h_irout[2];
    c->gir_rho_p = c->h_irout[0];
    c->gir_rho_d = c->h_irout[1];
    c->gir_kkt = kkt;
    if (!std::isfinite(kkt)) {
      launch_raise(c->d_status, FLAG_NONFINITE, s);
      break;
    }
    if (kkt <= tol) break;
    if (sw > 0 && !(kkt < 0.5 * prev)) {
      if (kkt <= 10.0 * tol) c->gir_stalled = 1;
      else launch_raise(c->d_status, FLAG_NOTCONV, s);
      break;
    }
    if (last) {
      launch_raise(c->d_status, FLAG_NOTCONV, s);
      break;
    }
    prev = kkt;
    TreeArgs tc = ta;
    tc.u = c->d_uc;
    tc.cc = c->d_cc;
    tc.glam = c->d_dlam;
    tc.f32 = 1;
    launch_tree(tc, c->d_gj, (int)c->tbody.size(), c->tc_rounds.data(), ((int)c->tc_rounds.size() - 1) / TC_NSEG,
                c->tree_split, c->tree_order, c->npath ? &c->pplan : nullptr, s);
    launch_gapply(c->gb0, c->gb1, c->d_inc_off, c->d_inc, c->d_gl, c->d_dlam, c->d_Rg, c->d_uc, c->ns,
                  c->d_shp, c->d_hinv, c->d_q[b], c->d_q[b], c->d_qd[b], h, 1, c->d_status, c->d_jrows, 0,
                  nullptr, c->opt.body_solve, 0, s);
    launch_lam_add(5 * (int64_t)mg, c->d_glam, c->d_dlam, c->d_status, s);
    ++c->gir_sweeps;
  }
  return hipGetLastError();
}

// Launch sequence of one step reading state buffer a and writing buffer b.
// The step index lives in device memory (begin_step), so this sequence can
// be captured once and replayed.
template <typename Timer>
hipError_t issue_step(mabd_ctx *c, double h, int a, int b, Timer &tm) {
  hipStream_t s = c->stream;
  const double *g = c->opt.gravity;
  const bool diag = (c->opt.diagnostics & 1) != 0 && c->d_dpart;
  launch_begin_step(c->d_status, s);
  if (!c->chains.empty()) {
    ChainArgs ca = chain_args(c, h, a, b);
    const int ntl = (int)c->tiles.size(), tt = c->tile_threads;
    const bool pk = c->tile_pack;
    // one chain solve: tile reduction, interface solve, tile back-substitution
    auto solve = [&](int mode) {
      const double *irs = mode == 2 ? c->d_ir : nullptr;
      tm.run(0, [&] { launch_chain_reduce(ca, ntl, tt, pk, mode, s); });
      tm.run(1, [&] {
        launch_chain_group(false, c->d_chains, c->d_groups, (int)c->groups.size(), c->d_tilerec,
                           c->d_grouprec, c->d_xtop, c->d_xg, c->d_gfac, c->d_gcount, c->d_status, 0,
                           irs, s);
        if (!c->top_in_group)
          launch_chain_global(c->d_chains, (int)c->chains.size(), c->d_grouprec, c->d_grow,
                              c->d_xtop, c->d_status, 0, irs, s);
        launch_chain_group(true, c->d_chains, c->d_groups, (int)c->groups.size(), c->d_tilerec,
                           c->d_grouprec, c->d_xtop, c->d_xg, c->d_gfac, c->d_gcount, c->d_status, 0,
                           irs, s);
      });
      tm.run(2, [&] { launch_chain_apply(ca, ntl, tt, pk, mode, s); });
    };
    if (c->opt.precision == 0) {
      solve(0);
    } else {
      // form 1: FP32 body/assembly solve, then FP64 KKT residual checks and
      // correction sweeps (each a solve with the residual as right-hand side)
      // until the KKT residual is <= kkt_tol
      launch_chain_ir_reset(c->d_ir, s);
      solve(1);
      const int nsw = c->opt.ir_max_sweeps;
      for (int sw = 0; sw <= nsw; ++sw) {
        const int final_check = sw == nsw ? 1 : 0;
        tm.run(8, [&] {
          launch_chain_resid(ca, ntl, tt, s);
          launch_chain_ir_check(c->d_part, ntl, c->opt.kkt_tol, final_check, c->d_ir, c->d_status, s);
        });
        if (!final_check) solve(2);
      }
      tm.run(9, [&] {
        launch_chain_finish(c->d_q[a], c->d_dq, c->d_q[b], c->d_qd[b], c->ns, c->nchain_bodies, h,
                            c->d_status, s);
      });
    }
  }
  if (c->gb1 > c->gb0) {
    // bodies without joints take their back-projection in the body kernel,
    // except when every iteration's residual is kept (it copies the iterate
    // before the back-projection updates it)
    const bool fuse_free = !(diag && c->opt.newton_iters > 1);
    for (int it = 0; it < c->opt.newton_iters; ++it) {
      const double *qcur = it == 0 ? c->d_q[a] : c->d_q[b];
      tm.run(3, [&] {
        launch_gbody(c->gb0, c->gb1, qcur, c->d_q[a], c->d_qd[a], c->ns, c->d_shp, c->d_hinv,
                     c->d_shape, g, h, c->d_Rg, c->d_ug, c->d_status, 0, c->wr_on ? c->d_wr : nullptr,
                     c->opt.body_solve == 1 ? c->d_inc_off : nullptr, c->gen_ir ? 1 : 0,
                     fuse_free ? c->d_inc_off : nullptr, c->d_q[b], c->d_qd[b], it > 0 ? 1 : 0, nullptr, s);
      });
      tm.run(4, [&] {
        launch_gjoint((int)c->gj.size(), c->d_gj, qcur, c->d_Rg, c->ns, c->opt.hinge_grad, c->d_gl, s);
      });
      TreeArgs ta{};
      ta.comp_lvl = c->d_comp_lvl;
      ta.lvl_off = c->d_lvl_off;
      ta.tbody = c->d_tbody;
      ta.tpk = c->d_tpk;
      ta.tabs_off = c->d_tabs_off;
      ta.tabs = c->d_tabs;
      ta.gl = c->d_gl;
      ta.gt = c->d_gt;
      ta.u = c->d_ug;
      ta.ns = c->ns;
      ta.shp = c->d_shp;
      ta.hinv = c->d_hinv;
      ta.glam = c->d_glam;
      ta.status = c->d_status;
      ta.step = 0;
      ta.tne = c->d_tne;
      ta.foff = c->d_foff;
      ta.fac = c->d_fac;
      ta.ops = c->d_tc_ops;
      ta.crec = c->d_crec;
      ta.f32 = c->gen_ir ? 1 : 0;
      ta.jrows = c->d_jrows;
      tm.run(5, [&] {
        // paths beside the contraction rounds (whose tail rounds leave most
        // of the GPU idle); sequential when kernel groups are timed
        const bool fork = c->side && (c->opt.diagnostics & 2) == 0;
        struct Fork {
          mabd_ctx *c;
          const TreeArgs *ta;
          hipStream_t s;
        } fk{c, &ta, s};
        auto do_fork = [](void *p) {
          const Fork &f = *static_cast<Fork *>(p);
          (void)hipEventRecord(f.c->ev_fork, f.s);
          (void)hipStreamWaitEvent(f.c->side, f.c->ev_fork, 0);
          launch_path(*f.ta, f.c->pplan, f.c->side);
          (void)hipEventRecord(f.c->ev_join, f.c->side);
        };
        launch_tree(ta, c->d_gj, (int)c->tbody.size(), c->tc_rounds.data(),
                    ((int)c->tc_rounds.size() - 1) / TC_NSEG, c->tree_split, c->tree_order,
                    !fork && c->npath ? &c->pplan : nullptr, s, c->fork_round, fork ? +do_fork : nullptr, &fk);
        if (fork) (void)hipStreamWaitEvent(s, c->ev_join, 0);
        if (c->nloop > 0) {
          // loop-breaker Schur complement (Case III): the columns
          // S_AA^{-1} S_AD e_j by tree solves of the loop rows' increments
          // with zero constraint values, then the Schur system per component
          // and the tree joints' correction
          const int64_t ws = 5 * (int64_t)c->gj.size();
          TreeArgs tw = ta;
          tw.u = c->d_uloop;
          tw.zero_c = 1;
          for (int j = 0; j < c->loop_maxr; ++j) {
            launch_loop_inject(c->nloop, c->d_loff, c->d_lrow, j, c->d_gj, c->d_gl, c->d_shp, c->d_hinv, c->ns,
                               c->d_uloop, 1, s);
            tw.glam = c->d_wcol + (size_t)j * ws;
            launch_tree(tw, c->d_gj, (int)c->tbody.size(), c->tc_rounds.data(),
                        ((int)c->tc_rounds.size() - 1) / TC_NSEG, c->tree_split, c->tree_order, c->npath ? &c->pplan : nullptr, s);
            launch_loop_inject(c->nloop, c->d_loff, c->d_lrow, j, c->d_gj, c->d_gl, c->d_shp, c->d_hinv, c->ns,
                               c->d_uloop, 0, s);
          }
          launch_loop_schur(c->nloop, c->d_loff, c->d_lrow, c->d_gj, c->d_gl, c->d_ug, c->d_shp, c->d_hinv,
                            c->ns, c->d_inc_off, c->d_inc, c->d_jloop, c->d_wcol, ws, c->d_glam, c->d_lamD,
                            c->d_status, s);
          launch_loop_correct((int)c->gj.size(), c->d_jloop, c->d_loff, c->d_wcol, ws, c->d_lamD, c->d_glam,
                              c->d_status, s);
        }
      });
      if (c->ngraph > 0) {
        PcgArgs pa{};
        pa.nb = c->gb1 - c->gb0;
        pa.b0 = c->gb0;
        pa.mj = (int)c->gj.size();
        pa.jmask = c->d_jmask;
        pa.bmask = c->d_bmask;
        pa.J = c->d_gj;
        pa.gl = c->d_gl;
        pa.ug = c->d_ug;
        pa.ns = c->ns;
        pa.shp = c->d_shp;
        pa.hinv = c->d_hinv;
        pa.inc_off = c->d_inc_off;
        pa.inc = c->d_inc;
        pa.lam = c->d_glam;
        pa.r = c->d_pr_;
        pa.p = c->d_pp;
        pa.z = c->d_pz;
        pa.sp = c->d_psp;
        pa.bv = c->d_pbv;
        pa.dinv = c->d_dinv;
        pa.zb = c->d_zb;
        pa.partial = c->d_partial;
        pa.tol = c->opt.kkt_tol;
        pa.max_iters = c->opt.max_iters;
        pa.warm = (c->opt.warm_start == 1 && c->warm_valid) ? 1 : 0;
        pa.iters_out = c->d_pcg_it;
        pa.res_out = c->d_pcg_res;
        pa.status = c->d_status;
        pa.step = 0;
        hipError_t pe = hipSuccess;
        if (c->pcg_ball) {
          PcgBallArgs pb = make_ball_args(c, pa.tol, pa.max_iters, pa.warm);
          tm.run(7, [&] { pe = run_pcg_ball(c, pb, s); });
        } else {
          tm.run(7, [&] { pe = launch_pcg(pa, c->pcg_blocks, s); });
        }
        if (pe != hipSuccess) return pe;
      }
      // diagnostics with several Newton iterations: the residual of every
      // iteration, from its own iterate and increment (the update below
      // overwrites the iterate in place, so it is saved first)
      const bool dg_it = diag && c->opt.newton_iters > 1;
      if (dg_it && it > 0) {
        hipError_t ce = hipMemcpyAsync(c->d_qit, c->d_q[b], (size_t)12 * c->ns * sizeof(double),
                                       hipMemcpyDeviceToDevice, s);
        if (ce != hipSuccess) return ce;
      }
      tm.run(6, [&] {
        launch_gapply(c->gb0, c->gb1, c->d_inc_off, c->d_inc, c->d_gl, c->d_glam, c->d_Rg, c->d_ug,
                      c->ns, c->d_shp, c->d_hinv, qcur, c->d_q[b], c->d_qd[b], h, it > 0 ? 1 : 0,
                      c->d_status, c->d_jrows, 0, dg_it ? c->d_dqit : nullptr, c->opt.body_solve,
                      fuse_free ? 1 : 0, s);
      });
      if (c->gen_ir) {
        hipError_t re = hipSuccess;
        tm.run(8, [&] { re = generic_refine(c, h, a, b, ta); });
        if (re != hipSuccess) return re;
      }
      if (dg_it) {
        const int slot = std::min(it, MABD_NEWTON_DIAG - 1);
        issue_residual(c, h, a, b, it > 0 ? c->d_qit : c->d_q[a], c->d_dqit, 1.0, c->d_dpart,
                       c->d_diag + 5 * (1 + slot));
        if (it == c->opt.newton_iters - 1) {
          hipError_t ce = hipMemcpyAsync(c->d_diag, c->d_diag + 5 * (1 + slot), 5 * sizeof(double),
                                         hipMemcpyDeviceToDevice, s);
          if (ce != hipSuccess) return ce;
        }
      }
    }
  }
  // diagnostics with one Newton iteration: the residual of the whole step
  // (chains and generic components), its increment being h times the new
  // velocity
  if (diag && c->opt.newton_iters == 1)
    issue_residual(c, h, a, b, c->d_q[a], c->d_qd[b], h, c->d_dpart, c->d_diag);
  return hipGetLastError();
}

struct NoTimer {
  template <typename F>
  void run(int, F &&f) { f(); }
};

// contexts large enough for the autotuner to time their schedules
constexpr int TUNE_MIN_ROWS = 20000;
bool tune_chain(const mabd_ctx *c) { return c->nchain_rows >= TUNE_MIN_ROWS; }
bool tune_tree(const mabd_ctx *c) { return (int)c->tbody.size() >= TUNE_MIN_ROWS && c->ngraph == 0; }

// Times the whole step for every chain tile form, then for every tree
// schedule, and keeps the fastest of each.  Every timed step reads the
// current state and writes only the scratch buffer, so the state does not
// advance.
hipError_t autotune(mabd_ctx *c, double h) {
  hipStream_t s = c->stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return hipErrorUnknown;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return hipErrorUnknown; }
  NoTimer nt;
  hipError_t e = hipSuccess;
  // one untimed step, then the mean of three
  auto time_step = [&](float &ms) {
    launch_reset_status(c->d_status, s);
    e = issue_step(c, h, c->cur, 1 - c->cur, nt);
    if (e != hipSuccess) return;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < 3; ++r) issue_step(c, h, c->cur, 1 - c->cur, nt);
    (void)hipEventRecord(e1, s);
    e = hipEventSynchronize(e1);
    if (e == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
  };
  if (tune_chain(c)) {
    int best = c->tile_threads;
    bool best_pack = c->tile_pack;
    float best_ms = 1e30f;
    const std::pair<int, bool> cand[] = {{64, true}, {64, false}, {128, false}, {256, false}};
    for (const auto &cv : cand) {
      e = build_tiles(c, cv.first, cv.second);
      if (e != hipSuccess) break;
      float ms = 0.f;
      time_step(ms);
      if (e != hipSuccess) break;
      if (ms < best_ms) { best_ms = ms; best = cv.first; best_pack = cv.second; }
    }
    if (e == hipSuccess) e = build_tiles(c, best, best_pack);
  }
  if (e == hipSuccess && tune_tree(c)) {
    const std::pair<int, int> cand[] = {{6000, 0}, {1500, 0}, {INT_MAX, 0}, {6000, 1}, {1500, 1}, {INT_MAX, 1}};
    std::pair<int, int> best = cand[0];
    float best_ms = 1e30f;
    for (const auto &cv : cand) {
      c->tree_split = cv.first;
      c->tree_order = cv.second;
      float ms = 0.f;
      time_step(ms);
      if (e != hipSuccess) break;
      if (ms < best_ms) { best_ms = ms; best = cv; }
    }
    c->tree_split = best.first;
    c->tree_order = best.second;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

// Tuning cache: the key names the device and the shape of the schedules
// (chain rows and count, tree slots and an FNV-1a hash of the contraction
// rounds' operation offsets); the value is tile threads, packed, tree split
// threshold and tree class order.
std::string tune_key(const mabd_ctx *c) {
  int dev = 0;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  for (char &ch : arch)
    if (ch == ' ' || ch == '=') ch = '_';
  uint64_t hsh = 1469598103934665603ull;
  for (int32_t v : c->tc_rounds) {
    uint32_t u = (uint32_t)v;
    for (int b = 0; b < 4; ++b) {
      hsh ^= (u >> (8 * b)) & 0xffu;
      hsh *= 1099511628211ull;
    }
  }
  char buf[256];
  std::snprintf(buf, sizeof buf, "mabd1 %s cu%d chain %lld/%zu tree %zu/%016llx", arch.c_str(), cus,
                (long long)c->nchain_rows, c->chains.size(), c->tbody.size(), (unsigned long long)hsh);
  return buf;
}

// the cached choices for this context, if the file has its key
bool tune_cache_read(const mabd_ctx *c, int &tt, int &pack, int &split, int &order) {
  if (c->tune_cache.empty()) return false;
  FILE *f = std::fopen(c->tune_cache.c_str(), "r");
  if (!f) return false;
  const std::string key = tune_key(c) + " = ";
  bool found = false;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    if (std::strncmp(line, key.c_str(), key.size()) != 0) continue;
    int a, b, d, e;
    if (std::sscanf(line + key.size(), "%d %d %d %d", &a, &b, &d, &e) == 4 &&
        (a == 64 || a == 128 || a == 256) && (b == 0 || b == 1) && d >= 0 && (e == 0 || e == 1)) {
      tt = a; pack = b; split = d; order = e;
      found = true;  // the last valid entry wins
    }
  }
  std::fclose(f);
  return found;
}

void tune_cache_append(const mabd_ctx *c) {
  if (c->tune_cache.empty()) return;
  FILE *f = std::fopen(c->tune_cache.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s = %d %d %d %d\n", tune_key(c).c_str(), c->tile_threads, c->tile_pack ? 1 : 0,
               c->tree_split, c->tree_order);
  std::fclose(f);
}

void drop_graphs(mabd_ctx *c) {
  for (int i = 0; i < 2; ++i)
    if (c->gexec[i]) {
      (void)hipGraphExecDestroy(c->gexec[i]);
      c->gexec[i] = nullptr;
    }
}

// capture one step per buffer parity; on any failure fall back to launches
void capture_graphs(mabd_ctx *c, double h) {
  NoTimer nt;
  for (int par = 0; par < 2; ++par) {
    hipGraph_t gr = nullptr;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) break;
    hipError_t e = issue_step(c, h, par, 1 - par, nt);
    hipError_t e2 = hipStreamEndCapture(c->stream, &gr);
    if (e != hipSuccess || e2 != hipSuccess || !gr) {
      if (gr) (void)hipGraphDestroy(gr);
      break;
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) break;
    c->gexec[par] = ex;
  }
  if (!c->gexec[0] || !c->gexec[1]) {
    drop_graphs(c);
    c->graph_failed = true;
    (void)hipGetLastError();
  }
}
}  // namespace

namespace {
// Reads the status of the steps issued since the status word was cleared
// (waiting for them) and settles the context: on a failure the state goes
// back to the buffer the failing step read (the steps after it did nothing),
// the step count stops before it and warm starts are withdrawn.  Returns the
// status of those steps; MABD_OK when nothing was pending.
mabd_status resolve(mabd_ctx *c) {
  if (!c->pending) return MABD_OK;
  const hipError_t e = hipEventSynchronize(c->pend_ev);
  c->pending = false;
  if (e != hipSuccess) {
    c->resid_ok = false;
    c->warm_valid = false;
    return fail(c, MABD_ERR_DEVICE, std::string("step: ") + hipGetErrorString(e));
  }
  if (c->ngraph > 0) {
    int32_t its;
    std::memcpy(&its, c->h_pcg + 1, sizeof its);
    c->stats.pcg_iters = its;
    c->stats.rho_d = c->h_pcg[0];
  }
  if (c->d_ir) {
    // FP64 KKT residual of the chains reached by the last step (form 1)
    c->stats.ir_sweeps = (int32_t)c->h_ir[1];
    c->stats.ir_stalled = c->h_ir[0] == 2.0 ? 1 : 0;
    c->stats.rho_p = c->h_ir[2];
    c->stats.rho_d = c->h_ir[3];
    c->stats.kkt = c->h_ir[4];
  }
  if (c->gen_ir) {
    // and of the generic components (the larger of the two where both exist)
    const bool both = c->d_ir != nullptr;
    c->stats.ir_sweeps = both ? std::max(c->stats.ir_sweeps, c->gir_sweeps) : c->gir_sweeps;
    c->stats.ir_stalled = (both && c->stats.ir_stalled) || c->gir_stalled ? 1 : 0;
    c->stats.rho_p = both ? std::max(c->stats.rho_p, c->gir_rho_p) : c->gir_rho_p;
    c->stats.rho_d = both ? std::max(c->stats.rho_d, c->gir_rho_d) : c->gir_rho_d;
    c->stats.kkt = both ? std::max(c->stats.kkt, c->gir_kkt) : c->gir_kkt;
  }
  for (int i = 0; i < MABD_NEWTON_DIAG; ++i) c->stats.kkt_newton[i] = -1.0;
  if ((c->opt.diagnostics & 1) && c->d_dpart) {
    // the FP64 KKT residual of the last step evaluated on the device
    const double *d = c->h_diag;
    c->stats.rho_p = d[0];
    c->stats.rho_d = d[1];
    c->stats.kkt = d[2];
    c->stats.c_ball = d[3];
    c->stats.c_hinge = d[4];
    if (c->opt.newton_iters == 1) {
      c->stats.kkt_newton[0] = d[2];
    } else {
      for (int i = 0; i < std::min(c->opt.newton_iters, MABD_NEWTON_DIAG); ++i)
        c->stats.kkt_newton[i] = d[5 * (1 + i) + 2];
    }
  }
  const uint32_t bits = c->h_status[0];
  if (bits) {
    const int f = (int)c->h_status[1];
    c->cur = (c->pend_cur0 + f) % 2;
    c->stats.steps_done += f;
    c->resid_ok = false;
    c->warm_valid = false;  // the failed step's multipliers are no start value
    c->stats.last_status = (bits & FLAG_GUARD)       ? MABD_ERR_DEVICE
                           : (bits & FLAG_NONFINITE) ? MABD_ERR_NONFINITE
                           : (bits & FLAG_SINGULAR)  ? MABD_ERR_SINGULAR
                                                     : MABD_ERR_NOT_CONVERGED;
    return fail(c, (mabd_status)c->stats.last_status,
                (bits & FLAG_GUARD)       ? "internal error: a tree operation exceeded its kernel's clique size"
                : (bits & FLAG_NONFINITE) ? "non-finite value or det A <= 0 during the step"
                : (bits & FLAG_SINGULAR)  ? "dual pivot block not positive definite"
                : c->d_ir                 ? "KKT residual above kkt_tol (PCG iteration cap, or "
                                            "precision-1 refinement out of sweeps or stalled)"
                                          : "PCG reached max_iters above kkt_tol");
  }
  c->stats.steps_done += c->pend_steps;
  c->stats.last_status = MABD_OK;
  c->warm_valid = true;
  return MABD_OK;
}

// The FP64 KKT residual of the last completed step (one Newton iteration),
// evaluated with the partial records in `part` (diag_nblk(c) of them),
// copied to out[0..4]; synchronises the stream.
mabd_status residual_into(mabd_ctx *c, double *part, double *out) {
  hipStream_t s = c->stream;
  const int a = 1 - c->cur, b = c->cur;
  issue_residual(c, c->h_last, a, b, c->d_q[a], c->d_qd[b], c->h_last, part, c->d_diag);
  hipError_t e = hipMemcpyAsync(c->h_diag, c->d_diag, 5 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, std::string("residual: ") + hipGetErrorString(e));
  for (int i = 0; i < 5; ++i) out[i] = c->h_diag[i];
  return MABD_OK;
}
}  // namespace

extern "C" {

mabd_status mabd_step(mabd_ctx *c, double h, int32_t nsteps) {
  if (!c) return MABD_ERR_INVALID_ARG;
  if (!(h > 0.0) || !std::isfinite(h)) return fail(c, MABD_ERR_INVALID_ARG, "h must be > 0");
  if (nsteps < 1) return fail(c, MABD_ERR_INVALID_ARG, "n must be >= 1");
  hipStream_t s = c->stream;
  // a failure of earlier steps whose status has already arrived is reported
  // now, before any new step is issued (no wait)
  if (c->pending && hipEventQuery(c->pend_ev) == hipSuccess) {
    const mabd_status st = resolve(c);
    if (st != MABD_OK) return st;
  }
  if (h != c->h_last) {
    launch_prefactor(c->d_shape, c->nshape, h, c->d_hinv, s);
    c->h_last = h;
    drop_graphs(c);
  }
  if (c->opt.autotune && !c->tuned && (tune_chain(c) || tune_tree(c))) {
    const mabd_status st = resolve(c);  // tuning clears the status word
    if (st != MABD_OK) return st;
    hipError_t te = autotune(c, h);
    if (te != hipSuccess) return fail(c, MABD_ERR_DEVICE, std::string("autotune: ") + hipGetErrorString(te));
    c->tuned = true;
    c->tune_source = 1;
    tune_cache_append(c);
    drop_graphs(c);
  }
  PhaseTimer tm(c);
  if (!c->pending) {
    launch_reset_status(c->d_status, s);
    c->pend_cur0 = c->cur;
    c->pend_steps = 0;
  }
  bool graph = c->opt.use_graph && c->ngraph == 0 && !c->gen_ir && !tm.on && !c->graph_failed;
  if (graph && !c->gexec[0]) capture_graphs(c, h);
  graph = graph && c->gexec[0] && c->gexec[1];
  c->stats.graph_replay = graph ? 1 : 0;
  c->stats.tile_threads = c->tile_threads;
  c->stats.tile_packed = c->tile_pack ? 1 : 0;
  c->stats.tree_split = c->tree_split;
  c->stats.tree_order = c->tree_order;
  c->stats.tune_source = c->tune_source;
  for (int st = 0; st < nsteps; ++st) {
    const int a = c->cur, b = 1 - c->cur;
    hipError_t le;
    if (graph) le = hipGraphLaunch(c->gexec[a], s);
    else le = issue_step(c, h, a, b, tm);
    if (le != hipSuccess) return fail(c, MABD_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(le));
    c->cur = b;
  }
  c->pend_steps += nsteps;
  c->resid_ok = true;  // withdrawn if the status read finds a failure
  // status words and results are copied now and read when a later call
  // needs them (resolve)
  hipError_t e = hipMemcpyAsync(c->h_status, c->d_status, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && c->d_ir)
    e = hipMemcpyAsync(c->h_ir, c->d_ir, 6 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && c->ngraph > 0) {
    e = hipMemcpyAsync(c->h_pcg, c->d_pcg_res, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->h_pcg + 1, c->d_pcg_it, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess && (c->opt.diagnostics & 1) && c->d_dpart)
    e = hipMemcpyAsync(c->h_diag, c->d_diag, DIAG_VALUES * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventRecord(c->pend_ev, s);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, std::string("step: ") + hipGetErrorString(e));
  c->pending = true;
  // networks are solved under host control and kernel timing needs the
  // events: those steps have synchronised already, so read the status now
  if (c->ngraph > 0 || c->gen_ir || tm.on) {
    const mabd_status st = resolve(c);
    tm.collect();
    return st;
  }
  return MABD_OK;
}

mabd_status mabd_state_device(const mabd_ctx *cc, void *q_dev, void *qd_dev) {
  mabd_ctx *c = const_cast<mabd_ctx *>(cc);
  if (!c) return MABD_ERR_INVALID_ARG;
  hipStream_t s = c->stream;
  // with steps in flight the kernel itself picks the last good buffer
  launch_gather_state(c->nd, c->d_sol2in, c->d_q, c->d_qd, c->cur, c->pend_cur0,
                      c->pending ? c->d_status : nullptr, c->ns, (double *)q_dev, (double *)qd_dev, s);
  launch_write_pinned((int)c->pin_idx.size(), c->d_pin_idx, c->d_pin_q0, (double *)q_dev,
                      (double *)qd_dev, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, hipGetErrorString(e));
  return MABD_OK;
}

mabd_status mabd_state(const mabd_ctx *cc, double *q, double *qd) {
  mabd_ctx *c = const_cast<mabd_ctx *>(cc);
  if (!c) return MABD_ERR_INVALID_ARG;
  const size_t n12 = (size_t)12 * c->n;
  double *tq = c->d_tmp, *tqd = c->d_tmp + n12;
  mabd_status st = mabd_state_device(c, tq, tqd);
  if (st != MABD_OK) return st;
  hipError_t e = hipSuccess;
  if (q && n12) e = hipMemcpyAsync(q, tq, n12 * 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && qd && n12) e = hipMemcpyAsync(qd, tqd, n12 * 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, hipGetErrorString(e));
  // the state copied is the last completed step's; a failure of the steps
  // in flight is reported here
  return resolve(c);
}

mabd_status mabd_set_state(mabd_ctx *c, const double *q, const double *qd) {
  if (!c || !q || !qd) return MABD_ERR_INVALID_ARG;
  const size_t n12 = (size_t)12 * c->n;
  if (!finite_all(q, n12) || !finite_all(qd, n12)) return fail(c, MABD_ERR_INVALID_ARG, "state not finite");
  for (int s = 0; s < c->nd; ++s) {
    const double *qq = q + 12 * (size_t)c->sol2in[s];
    double A[9] = {qq[0], qq[3], qq[6], qq[1], qq[4], qq[7], qq[2], qq[5], qq[8]};
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                 A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(det > 0)) return fail(c, MABD_ERR_INVALID_ARG, "det A <= 0 in the new state");
  }
  // settle steps in flight first (a failure among them stays in the stats);
  // the new state replaces whatever they left
  (void)resolve(c);
  c->warm_valid = false;  // the multipliers belong to another state
  c->resid_ok = false;
  double *tq = c->d_tmp, *tqd = c->d_tmp + n12;
  hipError_t e = hipSuccess;
  if (n12) e = hipMemcpyAsync(tq, q, n12 * 8, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && n12) e = hipMemcpyAsync(tqd, qd, n12 * 8, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) {
    launch_scatter_state(c->nd, c->d_sol2in, tq, tqd, c->d_q[c->cur], c->d_qd[c->cur], c->ns, c->stream);
    e = hipStreamSynchronize(c->stream);
  }
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, hipGetErrorString(e));
  return MABD_OK;
}

mabd_status mabd_set_wrenches(mabd_ctx *c, const double *w) {
  if (!c) return MABD_ERR_INVALID_ARG;
  (void)resolve(c);  // a failure among steps in flight stays in the stats
  if (!w) {
    if (c->wr_on) drop_graphs(c);  // the step launches change
    if (c->wr_on) c->resid_ok = false;
    c->wr_on = false;
    return MABD_OK;
  }
  const size_t n6 = (size_t)6 * c->n;
  if (!finite_all(w, n6)) return fail(c, MABD_ERR_INVALID_ARG, "wrench not finite");
  if (!c->d_wr) {
    hipError_t e = dalloc(c, &c->d_wr, 6 * (size_t)c->ns);
    if (e != hipSuccess) return fail(c, MABD_ERR_OOM, "wrench buffer");
  }
  // solver order, SoA; pinned bodies are not in the solver order
  std::vector<double> hw(6 * (size_t)c->ns, 0.0);
  for (int s = 0; s < c->nd; ++s)
    for (int k = 0; k < 6; ++k) hw[(size_t)k * c->ns + s] = w[6 * (size_t)c->sol2in[s] + k];
  hipError_t e = hipMemcpyAsync(c->d_wr, hw.data(), hw.size() * 8, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, hipGetErrorString(e));
  if (!c->wr_on) drop_graphs(c);
  c->wr_on = true;
  c->resid_ok = false;  // the last step ran with other loads
  return MABD_OK;
}

mabd_status mabd_multipliers(const mabd_ctx *cc, double *lam) {
  mabd_ctx *c = const_cast<mabd_ctx *>(cc);
  if (!c || !lam) return MABD_ERR_INVALID_ARG;
  const mabd_status rs = resolve(c);
  if (rs != MABD_OK) return rs;
  std::vector<double> cl(3 * (size_t)c->nchain_rows), gl(5 * c->gj.size());
  hipError_t e = hipSuccess;
  if (!cl.empty()) e = hipMemcpyAsync(cl.data(), c->d_clam, cl.size() * 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && !gl.empty())
    e = hipMemcpyAsync(gl.data(), c->d_glam, gl.size() * 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, hipGetErrorString(e));
  for (int r = 0; r < c->nchain_rows; ++r) {
    const int k = c->crow_joint[r];
    for (int i = 0; i < 3; ++i) lam[c->jrow_off[k] + i] = cl[3 * (size_t)r + i];
  }
  for (size_t gk = 0; gk < c->gj.size(); ++gk) {
    const int k = c->gj_in[gk];
    const int rk = joint_rows(c->jtype[k]);
    for (int i = 0; i < rk; ++i) lam[c->jrow_off[k] + i] = gl[5 * gk + i];
  }
  return MABD_OK;
}

mabd_status mabd_residual(mabd_ctx *c, double *out) {
  if (!c || !out) return MABD_ERR_INVALID_ARG;
  const mabd_status rs = resolve(c);
  if (rs != MABD_OK) return rs;
  if (!c->resid_ok)
    return fail(c, MABD_ERR_INVALID_ARG,
                "no completed step to check: a step must follow create, set_state, set_wrenches "
                "and the learned-start calls");
  if (c->opt.newton_iters != 1)
    return fail(c, MABD_ERR_INVALID_ARG,
                "newton_iters > 1: the iterates are not kept; diagnostics bit 0 reports every iteration");
  if (!c->d_dpart) {
    // partial records, kept until mabd_destroy
    hipError_t e = dalloc(c, &c->d_dpart, (size_t)DIAG_PART * diag_nblk(c));
    if (e != hipSuccess) return fail(c, MABD_ERR_OOM, "residual partials");
  }
  return residual_into(c, c->d_dpart, out);
}

mabd_status mabd_residual_noalloc(mabd_ctx *c, double *out_dev) {
  if (!c || !out_dev) return MABD_ERR_INVALID_ARG;
  const int64_t nb = diag_nblk(c);
  if (nb > resid_static_blocks())
    return fail(c, MABD_ERR_INVALID_ARG,
                "the assembly needs " + std::to_string(nb) + " partial records, the fixed scratch holds " +
                    std::to_string(resid_static_blocks()) + ": use mabd_residual");
  if (!c->resid_ok)
    return fail(c, MABD_ERR_INVALID_ARG,
                "no completed step to check: a step must follow create, set_state, set_wrenches "
                "and the learned-start calls");
  if (c->opt.newton_iters != 1)
    return fail(c, MABD_ERR_INVALID_ARG, "newton_iters > 1: the iterates are not kept");
  if (!c->d_rscratch) return fail(c, MABD_ERR_DEVICE, "fixed residual scratch unavailable");
  const int a = 1 - c->cur, b = c->cur;
  issue_residual(c, c->h_last, a, b, c->d_q[a], c->d_qd[b], c->h_last, c->d_rscratch, out_dev);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, std::string("residual: ") + hipGetErrorString(e));
  return MABD_OK;
}

mabd_status mabd_twists(const mabd_ctx *cc, double *V) {
  mabd_ctx *c = const_cast<mabd_ctx *>(cc);
  if (!c || !V) return MABD_ERR_INVALID_ARG;
  const mabd_status rs = resolve(c);
  if (rs != MABD_OK) return rs;
  const size_t n6 = (size_t)6 * c->n;
  double *t = c->d_tmp;  // 24 n doubles
  hipError_t e = n6 ? hipMemsetAsync(t, 0, n6 * 8, c->stream) : hipSuccess;
  if (e == hipSuccess) {
    launch_twists(c->nd, c->d_sol2in, c->d_q[c->cur], c->d_qd[c->cur], c->ns, t, c->stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess && n6) e = hipMemcpyAsync(V, t, n6 * 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, std::string("twists: ") + hipGetErrorString(e));
  return MABD_OK;
}

mabd_status mabd_joint_wrenches(const mabd_ctx *cc, double *W) {
  mabd_ctx *c = const_cast<mabd_ctx *>(cc);
  if (!c || !W) return MABD_ERR_INVALID_ARG;
  const mabd_status rs = resolve(c);
  if (rs != MABD_OK) return rs;
  if (!c->resid_ok)
    return fail(c, MABD_ERR_INVALID_ARG,
                "no completed step: a step must follow create, set_state, set_wrenches "
                "and the learned-start calls");
  if (c->opt.newton_iters != 1)
    return fail(c, MABD_ERR_INVALID_ARG, "newton_iters > 1: the last iterate's joint rows are not kept");
  const size_t n6 = (size_t)6 * c->n;
  double *t = c->d_tmp;
  const int a = 1 - c->cur;  // the state the step started from
  hipError_t e = n6 ? hipMemsetAsync(t, 0, n6 * 8, c->stream) : hipSuccess;
  if (e == hipSuccess) {
    launch_joint_wrenches(c->d_chains, (int)c->chains.size(), c->nchain_bodies, c->d_pl, c->d_pr, c->d_flag,
                          std::max(c->nchain_rows, 1), c->d_clam, c->gb0, c->gb1, c->d_Rg, c->d_inc_off,
                          c->d_inc, c->d_gj, c->d_gl, c->d_glam, c->d_q[a], c->ns, c->d_sol2in, t,
                          c->stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess && n6) e = hipMemcpyAsync(W, t, n6 * 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, std::string("joint wrenches: ") + hipGetErrorString(e));
  return MABD_OK;
}

mabd_status mabd_stats(const mabd_ctx *cc, mabd_step_stats *st) {
  mabd_ctx *c = const_cast<mabd_ctx *>(cc);
  if (!c || !st) return MABD_ERR_INVALID_ARG;
  (void)resolve(c);  // the outcome goes to st->last_status
  *st = c->stats;
  return MABD_OK;
}

int32_t mabd_gnn_size(void) { return GNN_NPARAM; }

mabd_status mabd_gnn_init(mabd_ctx *c, uint64_t seed) {
  mabd_status st = gnn_check(c, false);
  if (st != MABD_OK) return st;
  hipError_t e = gnn_alloc(c);
  if (e != hipSuccess) return fail(c, e == hipErrorOutOfMemory ? MABD_ERR_OOM : MABD_ERR_DEVICE, hipGetErrorString(e));
  std::vector<float> P;
  gnn_init_params(P, seed);
  e = gnn_set_params(c, P.data());
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, hipGetErrorString(e));
  return MABD_OK;
}

mabd_status mabd_gnn_params(mabd_ctx *c, float *get, const float *set, int32_t n) {
  mabd_status st = gnn_check(c, set == nullptr);
  if (st != MABD_OK) return st;
  if (n != GNN_NPARAM) return fail(c, MABD_ERR_INVALID_ARG, "n must equal mabd_gnn_size()");
  hipError_t e = hipSuccess;
  if (set) {
    e = gnn_alloc(c);
    if (e == hipSuccess) e = gnn_set_params(c, set);
  }
  if (e == hipSuccess && get)
    e = hipMemcpy(get, c->gb.params, GNN_NPARAM * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, hipGetErrorString(e));
  return MABD_OK;
}

mabd_status mabd_gnn_grad(mabd_ctx *c, double h, float *grad, double *loss) {
  mabd_status st = gnn_check(c, true);
  if (st != MABD_OK) return st;
  if (!(h > 0.0) || !std::isfinite(h)) return fail(c, MABD_ERR_INVALID_ARG, "h must be > 0");
  PcgBallArgs pb;
  hipError_t e = gnn_prepare(c, h, pb);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, hipGetErrorString(e));
  hipStream_t s = c->stream;
  launch_gnn_forward(pb, c->gb, c->warm_valid ? 1 : 0, s);
  launch_gnn_loss(pb, c->gb, s);
  launch_gnn_backward(pb, c->gb, s);
  e = hipMemcpyAsync(c->h_gsc, c->gb.sc + 2, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && grad)
    e = hipMemcpyAsync(grad, c->gb.grad, GNN_NPARAM * sizeof(float), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, hipGetErrorString(e));
  st = gnn_finish(c, "gnn_grad");
  if (st == MABD_OK && loss) *loss = c->h_gsc[0];
  return st;
}

mabd_status mabd_gnn_train(mabd_ctx *c, double h, int32_t iters, float lr, double *loss_first,
                           double *loss_last) {
  mabd_status st = gnn_check(c, true);
  if (st != MABD_OK) return st;
  if (!(h > 0.0) || !std::isfinite(h)) return fail(c, MABD_ERR_INVALID_ARG, "h must be > 0");
  if (iters < 0 || !(lr >= 0.0f) || !std::isfinite(lr)) return fail(c, MABD_ERR_INVALID_ARG, "iters, lr");
  PcgBallArgs pb;
  hipError_t e = gnn_prepare(c, h, pb);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, hipGetErrorString(e));
  hipStream_t s = c->stream;
  const int prev = c->warm_valid ? 1 : 0;
  for (int it = 0; it <= iters; ++it) {
    launch_gnn_forward(pb, c->gb, prev, s);
    launch_gnn_loss(pb, c->gb, s);
    if (it == 0) e = hipMemcpyAsync(c->h_gsc, c->gb.sc + 2, sizeof(double), hipMemcpyDeviceToHost, s);
    if (it == iters) {
      if (e == hipSuccess)
        e = hipMemcpyAsync(c->h_gsc + 1, c->gb.sc + 2, sizeof(double), hipMemcpyDeviceToHost, s);
      break;
    }
    launch_gnn_backward(pb, c->gb, s);
    launch_gnn_adam(c->gb, lr, ++c->gnn_t, s);
  }
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, hipGetErrorString(e));
  st = gnn_finish(c, "gnn_train");
  if (st == MABD_OK) {
    if (loss_first) *loss_first = c->h_gsc[0];
    if (loss_last) *loss_last = c->h_gsc[1];
  }
  return st;
}

mabd_status mabd_gnn_predict(mabd_ctx *c, double h, double *lam0) {
  mabd_status st = gnn_check(c, true);
  if (st != MABD_OK) return st;
  if (!(h > 0.0) || !std::isfinite(h) || !lam0) return fail(c, MABD_ERR_INVALID_ARG, "h, lam0");
  PcgBallArgs pb;
  hipError_t e = gnn_prepare(c, h, pb);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, hipGetErrorString(e));
  launch_gnn_forward(pb, c->gb, c->warm_valid ? 1 : 0, c->stream);
  launch_gnn_add_base(pb, c->gb, c->stream);
  std::vector<double> x(3 * (size_t)c->pb_nj);
  std::vector<int32_t> jid(c->pb_nj);
  e = hipMemcpyAsync(x.data(), pb.x, x.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(jid.data(), c->d_pb_jid, jid.size() * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, hipGetErrorString(e));
  st = gnn_finish(c, "gnn_predict");
  if (st != MABD_OK) return st;
  std::fill(lam0, lam0 + 3 * (size_t)c->m, 0.0);
  for (int j = 0; j < c->pb_nj; ++j) {
    const int k = c->gj_in[jid[j]];
    for (int r = 0; r < 3; ++r) lam0[3 * (size_t)k + r] = x[3 * (size_t)j + r];
  }
  return MABD_OK;
}

static const char GNN_MAGIC[8] = {'M', 'A', 'B', 'D', 'G', 'N', 'N', '1'};

mabd_status mabd_gnn_save(const mabd_ctx *cc, const char *path) {
  mabd_ctx *c = const_cast<mabd_ctx *>(cc);
  mabd_status st = gnn_check(c, true);
  if (st != MABD_OK) return st;
  if (!path) return fail(c, MABD_ERR_INVALID_ARG, "path");
  std::vector<float> P(GNN_NPARAM);
  hipError_t e = hipMemcpy(P.data(), c->gb.params, P.size() * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(c, MABD_ERR_DEVICE, hipGetErrorString(e));
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(c, MABD_ERR_INVALID_ARG, std::string("cannot open ") + path);
  const int32_t n = GNN_NPARAM;
  bool ok = std::fwrite(GNN_MAGIC, 1, 8, f) == 8 && std::fwrite(&n, sizeof n, 1, f) == 1 &&
            std::fwrite(P.data(), sizeof(float), P.size(), f) == P.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(c, MABD_ERR_INVALID_ARG, std::string("cannot write ") + path);
  return MABD_OK;
}

mabd_status mabd_gnn_load(mabd_ctx *c, const char *path) {
  mabd_status st = gnn_check(c, false);
  if (st != MABD_OK) return st;
  if (!path) return fail(c, MABD_ERR_INVALID_ARG, "path");
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(c, MABD_ERR_INVALID_ARG, std::string("cannot open ") + path);
  char magic[8];
  int32_t n = 0;
  std::vector<float> P(GNN_NPARAM);
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, GNN_MAGIC, 8) == 0 &&
            std::fread(&n, sizeof n, 1, f) == 1 && n == GNN_NPARAM &&
            std::fread(P.data(), sizeof(float), P.size(), f) == P.size();
  std::fclose(f);
  if (!ok) return fail(c, MABD_ERR_INVALID_ARG, std::string("not a weight file of this network: ") + path);
  for (float v : P)
    if (!std::isfinite(v)) return fail(c, MABD_ERR_INVALID_ARG, "weights not finite");
  hipError_t e = gnn_alloc(c);
  if (e == hipSuccess) e = gnn_set_params(c, P.data());
  if (e != hipSuccess) return fail(c, e == hipErrorOutOfMemory ? MABD_ERR_OOM : MABD_ERR_DEVICE, hipGetErrorString(e));
  return MABD_OK;
}

}  // extern "C"
