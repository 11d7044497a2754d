// C ABI of the D3M dual factorization and solution library (see d3m.h).
#include "../../include/d3m.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "launch.h"
#include "planner.h"
#include "static_ws.h"

using namespace d3m;

struct d3m_plan_s {
  PlanImpl p;
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace layout of one factor.
struct Layout {
  size_t L, LD, D, Linv, Ginv, Doff, ipiv, W, Z, X64, R64, P64, norms, ctrl, status, growth, counters, flags;
    size_t ftasks, fsucc, fcnt, stasks, ssucc, scnt, s2tasks, s2succ, s2cnt, sgtasks, sgsucc, sgcnt;
  size_t panels, pblocks, tiles, xsrc, iv;
  size_t kp, fills, rt, rptr, rblk, rsplit, nI, row0, prow0, perm, dkt, kg, kpart, knptr, knent;
  size_t total;
};

struct Tables {
  std::vector<KPlaceDev> kp, fills;
  std::vector<RTaskDev> rt;
  std::vector<int32_t> rptr;
  std::vector<RBlkDev> rblk;
  std::vector<int32_t> rsplit;
  std::vector<int32_t> nI;
  std::vector<int64_t> row0, prow0;
  std::vector<int32_t> perm;
  std::vector<DkTaskDev> dkt;
  std::vector<KPlaceDev> kg;  // reduced matrix out of panel storage (partial elimination)
  // ||K||_inf from the scatter's tile sums: per 32-row group of each
  // interface, the tile-sum vectors to add (KnormDev); kpart doubles of them
  std::vector<int32_t> kn_ptr;
  std::vector<int64_t> kn_ent;
  int64_t kpart = 0;
};

void make_tables(const PlanImpl& p, Tables& t) {
  // K placements with their tile-sum vectors (64 doubles per 32x32 tile),
  // and for every 32-row group of every interface the vectors that hold its
  // rows: row sums of the tiles whose rows are the group's, column sums of
  // the tiles whose columns are (placement order, then tile order)
  std::vector<int32_t> gbase(p.nb + 1, 0);
  for (int i = 0; i < p.nb; ++i) gbase[i + 1] = gbase[i] + (p.n[i] + 31) / 32;
  std::vector<std::vector<int64_t>> grp(gbase[p.nb]);
  for (auto& k : p.kplace) {
    const int tr = (k.rows + 31) / 32, tc = (k.cols + 31) / 32;
    t.kp.push_back({k.src, k.dst, k.rows, k.cols, k.ld_dst, k.trans, t.kpart, k.ri == k.ci && !k.trans, 0});
    for (int c = 0; c < tc; ++c)
      for (int r = 0; r < tr; ++r) {
        const int64_t v = t.kpart + (int64_t)(r + (int64_t)tr * c) * 64;
        grp[gbase[k.ri] + r].push_back(v);
        grp[gbase[k.ci] + c].push_back(v + 32);
      }
    t.kpart += (int64_t)tr * tc * 64;
  }
  t.kn_ptr.assign(1, 0);
  for (auto& g : grp) {
    t.kn_ent.insert(t.kn_ent.end(), g.begin(), g.end());
    t.kn_ptr.push_back((int32_t)t.kn_ent.size());
  }
  for (auto& f : p.fills) t.fills.push_back({0, f.dst, f.rows, f.cols, f.ld_dst, 0, -1, 0, 0});
  for (auto& k : p.kgather) t.kg.push_back({k.src, k.dst, k.rows, k.cols, k.ld_dst, k.trans, -1, 0, 0});
  t.nI = p.n;
  t.row0.assign(p.nb + 1, 0);
  for (int i = 0; i < p.nb; ++i) t.row0[i + 1] = t.row0[i] + p.n[i];
  t.prow0.assign(p.nb, 0);
  for (int i = 0; i < p.nb; ++i) t.prow0[i] = p.panels[p.pos[i]].prow0;
  t.perm.assign(p.N, 0);
  for (int i = 0; i < p.nb; ++i)
    for (int r = 0; r < p.n[i]; ++r) t.perm[t.prow0[i] + r] = (int32_t)(t.row0[i] + r);
  t.rptr.assign(p.nb + 1, 0);
  for (int i = 0; i < p.nb; ++i) {
    for (auto& b : p.rrow[i]) t.rblk.push_back({b.koff, b.J, b.mode});
    t.rptr[i + 1] = (int32_t)t.rblk.size();
  }
  // residual chunks: block z of row i starts at the first block whose
  // cumulative width reaches z/kResSplit of the row's width
  t.rsplit.assign((size_t)p.nb * (kResSplit + 1), 0);
  for (int i = 0; i < p.nb; ++i) {
    int64_t tot = 0;
    for (auto& b : p.rrow[i]) tot += p.n[b.J];
    int32_t* sp = &t.rsplit[(size_t)i * (kResSplit + 1)];
    int64_t cum = 0;
    int e = t.rptr[i], z = 1;
    sp[0] = t.rptr[i];
    for (auto& b : p.rrow[i]) {
      cum += p.n[b.J];
      ++e;
      while (z < kResSplit && cum * kResSplit >= tot * z) sp[z++] = e;
    }
    while (z <= kResSplit) sp[z++] = t.rptr[i + 1];
  }
  // residual / norm row tiles, largest work (rows x row length of K) first,
  // so that the hardware's in-order dispatch balances the tail
  std::vector<std::pair<int64_t, RTaskDev>> rts;
  for (int i = 0; i < p.nb; ++i) {
    int64_t len = 0;
    for (auto& b : p.rrow[i]) len += p.n[b.J];
    const Panel& P = p.panels[p.pos[i]];
    for (int c = 0; c < P.nt; ++c) {
      const Tile& T = p.tiles[P.tile0 + c];
      rts.push_back({(int64_t)T.sz * len, RTaskDev{i, T.r0, T.sz, 0}});
    }
  }
  std::stable_sort(rts.begin(), rts.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  for (auto& r : rts) t.rt.push_back(r.second);
  auto add_dk = [&](int64_t koff, int I, int J) {
    for (int r0 = 0; r0 < p.n[I]; r0 += kTileMax)
      for (int c0 = 0; c0 < p.n[J]; c0 += kTileMax)
        t.dkt.push_back({koff, I, J, r0, c0, std::min(kTileMax, p.n[I] - r0), std::min(kTileMax, p.n[J] - c0)});
  };
  for (int i = 0; i < p.nb; ++i) add_dk(p.koff[i], i, i);
  for (size_t k = 0; k < p.pairs.size(); ++k) add_dk(p.koff[p.nb + k], p.pairs[k][0], p.pairs[k][1]);
}

Layout make_layout(const PlanImpl& p, const Tables& t, int prec, int nrhs_max) {
  const size_t es = prec == 0 ? 16 : 8;
  Layout l;
  size_t o = 0;
  // 64 bytes of slack after every section: a paired complex64 load of an
  // odd last row reads one element past its operand
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + std::max<size_t>(bytes, 1) + 64); return at; };
  l.L = take(p.L_elems * es);
  l.LD = take(p.L_elems * es);
  l.D = take(p.N * es);
  l.Linv = take(p.Linv_elems * es);
  l.Ginv = take(p.Linv_elems * es);  // used with pivoting only
  l.Doff = take(p.N * es);
  l.ipiv = take(p.N * sizeof(int32_t));
  l.W = take((size_t)p.N * nrhs_max * es * (1 + kSolveSlots));  // b and its extra accumulators
  l.Z = take((size_t)p.N * nrhs_max * es);
  l.X64 = take((size_t)p.N * nrhs_max * 16);
  l.R64 = take((size_t)p.N * nrhs_max * 16);
  l.P64 = take((size_t)kResSplit * p.N * nrhs_max * 16);
  l.norms = take(3 * 128 * sizeof(double));
  l.ctrl = take(sizeof(IrCtrl));
  l.status = take(4 * sizeof(int32_t));
  l.growth = take(2 * p.nb * sizeof(float));
    l.counters = take(std::max({p.fdag.tasks.size(), p.sdag.tasks.size(), p.sdag2.tasks.size(), p.sdagg.tasks.size()}) *
                    sizeof(int32_t));
  l.flags = take(4 * sizeof(int32_t));
  l.ftasks = take(p.fdag.tasks.size() * sizeof(Task));
  l.fsucc = take(p.fdag.succ.size() * sizeof(int32_t));
  l.fcnt = take(p.fdag.npred.size() * sizeof(int32_t));
  l.stasks = take(p.sdag.tasks.size() * sizeof(Task));
  l.ssucc = take(p.sdag.succ.size() * sizeof(int32_t));
  l.scnt = take(p.sdag.npred.size() * sizeof(int32_t));
  l.s2tasks = take(p.sdag2.tasks.size() * sizeof(Task));
  l.s2succ = take(p.sdag2.succ.size() * sizeof(int32_t));
    l.s2cnt = take(p.sdag2.npred.size() * sizeof(int32_t));
  l.sgtasks = take(p.sdagg.tasks.size() * sizeof(Task));
  l.sgsucc = take(p.sdagg.succ.size() * sizeof(int32_t));
  l.sgcnt = take(p.sdagg.npred.size() * sizeof(int32_t));
  l.panels = take(p.panels.size() * sizeof(Panel));
  l.pblocks = take(p.pblocks.size() * sizeof(PBlock));
  l.tiles = take(p.tiles.size() * sizeof(Tile));
  l.xsrc = take(p.xsrc.size() * sizeof(XSrc));
  l.iv = take(sizeof(InstView));
  l.kp = take(t.kp.size() * sizeof(KPlaceDev));
  l.fills = take(t.fills.size() * sizeof(KPlaceDev));
  l.rt = take(t.rt.size() * sizeof(RTaskDev));
  l.rptr = take(t.rptr.size() * sizeof(int32_t));
  l.rblk = take(t.rblk.size() * sizeof(RBlkDev));
  l.rsplit = take(t.rsplit.size() * sizeof(int32_t));
  l.nI = take(t.nI.size() * sizeof(int32_t));
  l.row0 = take(t.row0.size() * sizeof(int64_t));
  l.prow0 = take(t.prow0.size() * sizeof(int64_t));
  l.perm = take(t.perm.size() * sizeof(int32_t));
  l.dkt = take(t.dkt.size() * sizeof(DkTaskDev));
  l.kg = take(t.kg.size() * sizeof(KPlaceDev));
  l.kpart = take(t.kpart * sizeof(double));
  l.knptr = take(t.kn_ptr.size() * sizeof(int32_t));
  l.knent = take(t.kn_ent.size() * sizeof(int64_t));
  l.total = o;
  return l;
}

int device_cus() {
  static int cus = -1;
  if (cus < 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
  }
  return cus;
}

}  // namespace

struct d3m_factor_s {
  const d3m_plan_s* plan = nullptr;
  int prec = 0;
  int nrhs_max = 0;
  char* ws = nullptr;
  size_t bytes = 0;
  d3m_options opt{};
  Layout lay{};
  Tables tab;
  hipStream_t last = nullptr;
  bool factored = false;
  int nworkers = 256;
  int red_nrhs = 0;  // right-hand sides of the last d3m_reduce's forward part (d3m_recover continues it)
  // bound to the library's static device array of device sdev (>= 0), as
  // generation sgen; a later static bind on that device invalidates it
  int sdev = -1;
  unsigned long long sgen = 0;
  // timing: event pairs around DAG launches, [0] factor, [1] solve
  static constexpr int kRing = 64;
  void* trace = nullptr;  // optional task trace buffer (caller-owned device memory)
  size_t trace_bytes = 0;
  std::vector<hipEvent_t> ev[2];
  int nev[2] = {0, 0};
  template <typename P> P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
  UserView uv() const {
    UserView u;
    u.n = at<int32_t>(lay.nI);
    u.row0 = at<int64_t>(lay.row0);
    u.prow0 = at<int64_t>(lay.prow0);
    u.rptr = at<int32_t>(lay.rptr);
    u.rblk = at<RBlkDev>(lay.rblk);
    u.rsplit = at<int32_t>(lay.rsplit);
    u.perm = at<int32_t>(lay.perm);
    u.N = plan->p.N;
    return u;
  }
  KnormDev kn() const {
    KnormDev k;
    k.part = at<double>(lay.kpart);
    k.ptr = at<int32_t>(lay.knptr);
    k.ent = at<int64_t>(lay.knent);
    k.ngroups = (int32_t)tab.kn_ptr.size() - 1;
    k.pad = 0;
    return k;
  }
  IrCtrl* ctrl() const { return at<IrCtrl>(lay.ctrl); }
  int32_t* stop() const { return &ctrl()->stop; }
  double* rmax() const { return at<double>(lay.norms); }
  double* xmax() const { return at<double>(lay.norms) + 128; }
  double* bmax() const { return at<double>(lay.norms) + 256; }
};

#define HIPCHK(x)                                  \
  do {                                             \
    if ((x) != hipSuccess) return D3M_ERR_HIP;     \
  } while (0)

namespace {

// which: 0 the factor DAG, 1 the solve DAG (with a partial elimination its
// forward part), 2 the backward part of a partial elimination's solve.  A
// solve whose right-hand sides give every group of the plan's grouped solve
// DAG at least 16 columns runs that one (3).
d3m_status run_dag(d3m_factor_s* f, int which, int nrhs, const int32_t* skip, hipStream_t s) {
  const PlanImpl& p = f->plan->p;
  const bool solve = which != 0;
  if (which == 1 && p.rhs_groups > 1 && !p.sdagg.tasks.empty() && nrhs >= 16 * p.rhs_groups) which = 3;
  const TaskDag& dag = which == 0 ? p.fdag : (which == 1 ? p.sdag : (which == 2 ? p.sdag2 : p.sdagg));
  const size_t tk[4] = {f->lay.ftasks, f->lay.stasks, f->lay.s2tasks, f->lay.sgtasks};
  const size_t sc[4] = {f->lay.fsucc, f->lay.ssucc, f->lay.s2succ, f->lay.sgsucc};
  const size_t cn[4] = {f->lay.fcnt, f->lay.scnt, f->lay.s2cnt, f->lay.sgcnt};
  DagArgs a;
  a.tasks = f->at<Task>(tk[which]);
  a.succ = f->at<int32_t>(sc[which]);
  a.rhs_groups = which == 3 ? p.rhs_groups : 1;
  a.counters = f->at<int32_t>(f->lay.counters);
  int32_t* flags = f->at<int32_t>(f->lay.flags);
  a.head = flags;
  a.abort_flag = flags + 1;
  a.skip = skip;
  a.inst = f->at<InstView>(f->lay.iv);
  a.ntask = (int32_t)dag.tasks.size();
  a.nrhs = nrhs;
  a.spin_limit_ns = 20LL * 1000 * 1000 * 1000;  // 20 s on one wait
  a.trace = nullptr;
  if (f->trace && (size_t)a.ntask * 32 <= f->trace_bytes / 2)
    a.trace = reinterpret_cast<int64_t*>(static_cast<char*>(f->trace) + (solve ? f->trace_bytes / 2 : 0));
    HIPCHK(launch_reset(a.counters, f->at<int32_t>(cn[which]), a.ntask, a.head, a.abort_flag, skip, s));
  const int w = solve ? 1 : 0;
  const bool timed = f->opt.timing && !skip && f->nev[w] < d3m_factor_s::kRing;
  if (timed) HIPCHK(hipEventRecord(f->ev[w][2 * f->nev[w]], s));
  HIPCHK(launch_dag(a, f->prec, f->nworkers, solve, s));
  if (timed) {
    HIPCHK(hipEventRecord(f->ev[w][2 * f->nev[w] + 1], s));
    f->nev[w]++;
  }
  return D3M_OK;
}

}  // namespace

extern "C" {

const char* d3m_status_string(d3m_status s) {
  switch (s) {
    case D3M_OK: return "ok";
    case D3M_ERR_ARG: return "invalid argument";
    case D3M_ERR_PATTERN: return "invalid block pattern or order";
    case D3M_ERR_WORKSPACE: return "workspace too small or misaligned";
    case D3M_ERR_STATE: return "call out of sequence";
    case D3M_ERR_HIP: return "HIP runtime error";
    case D3M_ERR_HANG: return "dependency wait exceeded the watchdog bound";
    case D3M_ERR_NORUNTIME: return "no usable gfx950 device";
    case D3M_ZERO_PIVOT: return "zero or non-finite pivot";
    case D3M_NONFINITE: return "non-finite value in the solution";
    case D3M_IR_NOCONV: return "iterative refinement did not converge";
  }
  return "unknown status";
}

int32_t d3m_device_ok(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return 0;
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  return std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
}

d3m_status d3m_analyze(int32_t nblk, const int32_t* blk_size, int64_t npair, const int32_t* pairs,
                       const int32_t* order, const int32_t* grid, const d3m_analyze_options* opt,
                       d3m_plan* out) {
  if (!out) return D3M_ERR_ARG;
  *out = nullptr;
  d3m_analyze_options o{};
  if (opt) o = *opt;
  d3m_plan_s* pl = new (std::nothrow) d3m_plan_s;
  if (!pl) return D3M_ERR_ARG;
  int err = 0;
    std::string msg = build_plan(pl->p, nblk, blk_size, npair, pairs, order, grid, o.tile, o.nworkers, o.sched,
                               o.nelim, o.solve_tile, o.merge, o.rhs_groups, &err);
  if (!msg.empty()) {
    delete pl;
    return (d3m_status)err;
  }
  *out = pl;
  return D3M_OK;
}

d3m_status d3m_plan_query(d3m_plan plan, d3m_plan_info* o) {
  if (!plan || !o) return D3M_ERR_ARG;
  const PlanImpl& p = plan->p;
  std::memset(o, 0, sizeof(*o));
  o->N = p.N;
  o->nblk = p.nb;
  o->npair = (int64_t)p.pairs.size();
  o->k_len = p.koff.back();
  o->fill_blocks = p.fill_blocks;
  o->L_blocks = p.L_blocks;
  o->nnz_L = p.nnz_L;
  o->nnz_K = p.nnz_K;
  o->etree_height = p.etree_height;
  o->max_S = p.max_S;
  o->ntask_factor = (int64_t)p.fdag.tasks.size();
  o->ntask_solve = (int64_t)p.sdag.tasks.size();
  o->ntiles = (int64_t)p.tiles.size();
  o->flops_diag = p.flops_diag;
  o->flops_trsm = p.flops_trsm;
  o->flops_update = p.flops_update;
  o->flops_factor = p.flops_diag + p.flops_trsm + p.flops_update;
  o->solve_flops_per_rhs = 16.0 * (double)p.nnz_L;
  o->sim_factor_us = p.fdag.makespan_us;
  return D3M_OK;
}

d3m_status d3m_plan_order(d3m_plan plan, int32_t* order) {
  if (!plan || !order) return D3M_ERR_ARG;
  std::copy(plan->p.order.begin(), plan->p.order.end(), order);
  return D3M_OK;
}

d3m_status d3m_plan_k_offsets(d3m_plan plan, int64_t* offsets) {
  if (!plan || !offsets) return D3M_ERR_ARG;
  std::copy(plan->p.koff.begin(), plan->p.koff.end(), offsets);
  return D3M_OK;
}

d3m_status d3m_plan_struct(d3m_plan plan, int32_t I, int32_t* S, int32_t* count) {
  if (!plan || !S || !count || I < 0 || I >= plan->p.nb) return D3M_ERR_ARG;
  const PlanImpl& p = plan->p;
  const auto& s = p.S[p.pos[I]];
  for (size_t u = 0; u < s.size(); ++u) S[u] = p.order[s[u]];
  *count = (int32_t)s.size();
  return D3M_OK;
}

d3m_status d3m_plan_check(d3m_plan plan, int64_t* nviolations) {
  if (!plan || !nviolations) return D3M_ERR_ARG;
  const PlanImpl& p = plan->p;
  if (p.facc.empty() || p.sacc.empty()) return D3M_ERR_STATE;  // too large to check
  int64_t a = check_dag(p.fdag, p.facc), b = check_dag(p.sdag, p.sacc);
    if (p.nelim > 0) {
    const int64_t c = p.sacc2.empty() ? -1 : check_dag(p.sdag2, p.sacc2);
    if (c < 0) b = -1;
    else b += c;
  }
  if (p.rhs_groups > 1) {
    const int64_t c = p.saccg.empty() ? -1 : check_dag(p.sdagg, p.saccg);
    if (c < 0) b = -1;
    else b += c;
  }
  if (a < 0 || b < 0) {
    *nviolations = -1;
    return D3M_ERR_STATE;
  }
  *nviolations = a + b;
  return D3M_OK;
}

void d3m_plan_destroy(d3m_plan plan) { delete plan; }

d3m_status d3m_workspace_bytes(d3m_plan plan, d3m_precision prec, int32_t nrhs_max, size_t* bytes) {
  if (!plan || !bytes || nrhs_max < 1 || nrhs_max > 128 || (prec != D3M_C128 && prec != D3M_C64_IR))
    return D3M_ERR_ARG;
  Tables t;
  make_tables(plan->p, t);
  *bytes = make_layout(plan->p, t, prec == D3M_C128 ? 0 : 1, nrhs_max).total;
  return D3M_OK;
}

d3m_status d3m_factor_bind(d3m_plan plan, d3m_precision prec, void* dev_ws, size_t bytes, int32_t nrhs_max,
                           const d3m_options* opt, d3m_factor* out) {
  return d3m::bind_factor(plan, prec, dev_ws, bytes, nrhs_max, opt, -1, 0, out);
}

}  // extern "C"

d3m_status d3m::bind_factor(d3m_plan plan, d3m_precision prec, void* dev_ws, size_t bytes, int32_t nrhs_max,
                            const d3m_options* opt, int sdev, unsigned long long sgen, d3m_factor* out) {
  if (!plan || !out || !dev_ws || nrhs_max < 1 || nrhs_max > 128 || (prec != D3M_C128 && prec != D3M_C64_IR))
    return D3M_ERR_ARG;
  *out = nullptr;
  if (reinterpret_cast<uintptr_t>(dev_ws) % kAlign) return D3M_ERR_WORKSPACE;
  d3m_factor_s* f = new (std::nothrow) d3m_factor_s;
  if (!f) return D3M_ERR_ARG;
  f->sdev = sdev;
  f->sgen = sgen;
  f->plan = plan;
  f->prec = prec == D3M_C128 ? 0 : 1;
  f->nrhs_max = nrhs_max;
  make_tables(plan->p, f->tab);
  f->lay = make_layout(plan->p, f->tab, f->prec, nrhs_max);
  if (bytes < f->lay.total) {
    delete f;
    return D3M_ERR_WORKSPACE;
  }
  f->ws = static_cast<char*>(dev_ws);
  f->bytes = bytes;
  if (opt) f->opt = *opt;
  if (f->opt.tol <= 0) f->opt.tol = 1e-10;
  if (f->opt.max_iter <= 0) f->opt.max_iter = 10;
  if (f->opt.max_iter > 30) f->opt.max_iter = 30;
  if (f->opt.growth_dmin <= 0) f->opt.growth_dmin = 1e-4;
  if (f->opt.growth_lmax <= 0) f->opt.growth_lmax = 1e2;
  f->nworkers = device_cus();
  const PlanImpl& p = plan->p;
  auto up = [&](size_t off, const void* src, size_t n) -> bool {
    if (n == 0) return true;
    return hipMemcpy(f->ws + off, src, n, hipMemcpyHostToDevice) == hipSuccess;
  };
  InstView iv{};
  iv.L = f->ws + f->lay.L;
  iv.LD = f->ws + f->lay.LD;
  iv.D = f->ws + f->lay.D;
  iv.Linv = f->ws + f->lay.Linv;
  iv.W = f->ws + f->lay.W;
  iv.Z = f->ws + f->lay.Z;
  iv.panels = f->at<Panel>(f->lay.panels);
  iv.pblocks = f->at<PBlock>(f->lay.pblocks);
  iv.tiles = f->at<Tile>(f->lay.tiles);
  iv.xsrc = f->at<XSrc>(f->lay.xsrc);
  iv.status = f->at<int32_t>(f->lay.status);
  iv.growth = f->at<float>(f->lay.growth);
  iv.nrhs = nrhs_max;
  iv.npanel = p.nb;
  iv.N = p.N;
  iv.gdmin = (float)f->opt.growth_dmin;
  iv.glmax = (float)f->opt.growth_lmax;
  iv.pivot = f->opt.pivot ? 1 : 0;
  iv.fallback = (f->opt.fallback < 0 || iv.pivot) ? 0 : 1;
  iv.Ginv = f->ws + f->lay.Ginv;
  iv.Doff = f->ws + f->lay.Doff;
  iv.ipiv = f->at<int32_t>(f->lay.ipiv);
  bool ok = up(f->lay.ftasks, p.fdag.tasks.data(), p.fdag.tasks.size() * sizeof(Task)) &&
            up(f->lay.fsucc, p.fdag.succ.data(), p.fdag.succ.size() * 4) &&
            up(f->lay.fcnt, p.fdag.npred.data(), p.fdag.npred.size() * 4) &&
            up(f->lay.stasks, p.sdag.tasks.data(), p.sdag.tasks.size() * sizeof(Task)) &&
            up(f->lay.ssucc, p.sdag.succ.data(), p.sdag.succ.size() * 4) &&
            up(f->lay.scnt, p.sdag.npred.data(), p.sdag.npred.size() * 4) &&
            up(f->lay.s2tasks, p.sdag2.tasks.data(), p.sdag2.tasks.size() * sizeof(Task)) &&
            up(f->lay.s2succ, p.sdag2.succ.data(), p.sdag2.succ.size() * 4) &&
                        up(f->lay.s2cnt, p.sdag2.npred.data(), p.sdag2.npred.size() * 4) &&
            up(f->lay.sgtasks, p.sdagg.tasks.data(), p.sdagg.tasks.size() * sizeof(Task)) &&
            up(f->lay.sgsucc, p.sdagg.succ.data(), p.sdagg.succ.size() * 4) &&
            up(f->lay.sgcnt, p.sdagg.npred.data(), p.sdagg.npred.size() * 4) &&
            up(f->lay.kg, f->tab.kg.data(), f->tab.kg.size() * sizeof(KPlaceDev)) &&
            up(f->lay.panels, p.panels.data(), p.panels.size() * sizeof(Panel)) &&
            up(f->lay.pblocks, p.pblocks.data(), p.pblocks.size() * sizeof(PBlock)) &&
            up(f->lay.tiles, p.tiles.data(), p.tiles.size() * sizeof(Tile)) &&
            up(f->lay.xsrc, p.xsrc.data(), p.xsrc.size() * sizeof(XSrc)) &&
            up(f->lay.iv, &iv, sizeof(iv)) &&
            up(f->lay.kp, f->tab.kp.data(), f->tab.kp.size() * sizeof(KPlaceDev)) &&
            up(f->lay.fills, f->tab.fills.data(), f->tab.fills.size() * sizeof(KPlaceDev)) &&
            up(f->lay.rt, f->tab.rt.data(), f->tab.rt.size() * sizeof(RTaskDev)) &&
            up(f->lay.rptr, f->tab.rptr.data(), f->tab.rptr.size() * 4) &&
            up(f->lay.rblk, f->tab.rblk.data(), f->tab.rblk.size() * sizeof(RBlkDev)) &&
            up(f->lay.rsplit, f->tab.rsplit.data(), f->tab.rsplit.size() * 4) &&
            up(f->lay.nI, f->tab.nI.data(), f->tab.nI.size() * 4) &&
            up(f->lay.row0, f->tab.row0.data(), f->tab.row0.size() * 8) &&
            up(f->lay.prow0, f->tab.prow0.data(), f->tab.prow0.size() * 8) &&
            up(f->lay.perm, f->tab.perm.data(), f->tab.perm.size() * 4) &&
            up(f->lay.dkt, f->tab.dkt.data(), f->tab.dkt.size() * sizeof(DkTaskDev)) &&
            up(f->lay.knptr, f->tab.kn_ptr.data(), f->tab.kn_ptr.size() * 4) &&
            up(f->lay.knent, f->tab.kn_ent.data(), f->tab.kn_ent.size() * 8);
  if (f->opt.timing) {
    for (int w = 0; w < 2; ++w) {
      f->ev[w].resize(2 * d3m_factor_s::kRing);
      for (auto& e : f->ev[w]) ok = ok && hipEventCreate(&e) == hipSuccess;
    }
  }
  // flags, status and refinement control start cleared
  ok = ok && hipMemset(f->ws + f->lay.flags, 0, 16) == hipSuccess &&
       hipMemset(f->ws + f->lay.ctrl, 0, sizeof(IrCtrl)) == hipSuccess &&
       hipMemset(f->ws + f->lay.status, 0, 16) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    delete f;
    return D3M_ERR_HIP;
  }
  *out = f;
  return D3M_OK;
}

namespace {
// a factor bound to the static array after which another factor was bound there
bool stale(const d3m_factor_s* f) { return f->sdev >= 0 && !d3m::static_ws_valid(f->sdev, f->sgen); }
}  // namespace

extern "C" {

d3m_status d3m_factorize(d3m_factor f, const void* dev_K, d3m_stream stream) {
  if (!f || !dev_K) return D3M_ERR_ARG;
  if (f->plan->p.nelim > 0) return D3M_ERR_STATE;  // a partial elimination: d3m_reduce
  if (stale(f)) return D3M_ERR_STATE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const PlanImpl& p = f->plan->p;
  HIPCHK(launch_prepare(f->at<int32_t>(f->lay.status), f->at<float>(f->lay.growth), p.nb, f->ctrl(), f->opt.tol,
                        f->opt.max_iter, s));
  HIPCHK(launch_scatter(dev_K, f->ws + f->lay.L, f->at<KPlaceDev>(f->lay.kp), (int)f->tab.kp.size(),
                        f->at<KPlaceDev>(f->lay.fills), (int)f->tab.fills.size(), f->at<double>(f->lay.kpart),
                        f->prec, s));
  HIPCHK(launch_knorm(f->kn(), f->ctrl(), s));
  d3m_status st = run_dag(f, 0, f->nrhs_max, nullptr, s);
  if (st != D3M_OK) return st;
  f->last = s;
  f->factored = true;
  return D3M_OK;
}

namespace {

d3m_status solve_impl(d3m_factor f, const void* K, const void* B, void* X, int nrhs, int64_t ld, hipStream_t s) {
  const PlanImpl& p = f->plan->p;
  const int64_t N = p.N;
  UserView uv = f->uv();
  IrCtrl* c = f->ctrl();
  // refinement bookkeeping reset (keeps ||K||)
  HIPCHK(launch_ir_reset(c, f->opt.tol, f->opt.max_iter, s));
  HIPCHK(launch_zero_f64(f->rmax(), 3 * 128, s));
  HIPCHK(launch_colmax(B, N, nrhs, ld, 0, f->bmax(), nullptr, s));
  const RTaskDev* rt = f->at<RTaskDev>(f->lay.rt);
  const int nrt = (int)f->tab.rt.size();
  void* W = f->ws + f->lay.W;
  void* X64 = f->ws + f->lay.X64;
  void* R64 = f->ws + f->lay.R64;
  if (f->prec == 0) {
    HIPCHK(launch_perm_in(B, ld, W, 0, uv, nrhs, nullptr, s));
    d3m_status st = run_dag(f, 1, nrhs, nullptr, s);
    if (st) return st;
    HIPCHK(launch_residual(K, B, ld, W, R64, f->ws + f->lay.P64, f->rmax(), uv, rt, nrt, nrhs, nullptr, s));
    HIPCHK(launch_colmax(W, N, nrhs, 0, 1, f->xmax(), nullptr, s));
    HIPCHK(launch_ir_check(c, f->rmax(), f->xmax(), f->bmax(), nrhs, 2, s));
    HIPCHK(launch_perm_out(W, X, ld, uv, nrhs, s));
    return D3M_OK;
  }
  const int64_t nel = N * nrhs;
  HIPCHK(launch_perm_in(B, ld, W, 1, uv, nrhs, nullptr, s));
  d3m_status st = run_dag(f, 1, nrhs, nullptr, s);
  if (st) return st;
  HIPCHK(launch_cvt_up(W, X64, nel, s));
  const int32_t* stop = f->stop();
  for (int it = 0; it <= f->opt.max_iter; ++it) {
    HIPCHK(launch_residual(K, B, ld, X64, R64, f->ws + f->lay.P64, f->rmax(), uv, rt, nrt, nrhs, stop, s));
    HIPCHK(launch_colmax(X64, N, nrhs, 0, 1, f->xmax(), stop, s));
    HIPCHK(launch_ir_check(c, f->rmax(), f->xmax(), f->bmax(), nrhs, it == f->opt.max_iter ? 1 : 0, s));
    if (f->opt.ir_host_sync) {
      int32_t h = 0;
      HIPCHK(hipMemcpyAsync(&h, stop, 4, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (h) break;
    }
    if (it == f->opt.max_iter) break;
    HIPCHK(launch_cvt_down(R64, W, nel, stop, s));
    st = run_dag(f, 1, nrhs, stop, s);
    if (st) return st;
    HIPCHK(launch_axpy_up(W, X64, nel, stop, s));
  }
  HIPCHK(launch_perm_out(X64, X, ld, uv, nrhs, s));
  return D3M_OK;
}

}  // namespace

d3m_status d3m_solve(d3m_factor f, const void* dev_K, const void* dev_B, void* dev_X, int32_t nrhs, int64_t ld,
                     d3m_stream stream) {
  if (!f || !dev_K || !dev_B || !dev_X || nrhs < 1 || nrhs > f->nrhs_max || ld < f->plan->p.N) return D3M_ERR_ARG;
  if (!f->factored || stale(f) || f->plan->p.nelim > 0) return D3M_ERR_STATE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  d3m_status st = solve_impl(f, dev_K, dev_B, dev_X, nrhs, ld, s);
  f->last = s;
  return st;
}

d3m_status d3m_adjoint(d3m_factor f, const void* dev_K, const void* dev_X, const void* dev_G, void* dev_Lambda,
                       void* dev_dK, int32_t nrhs, int64_t ld, d3m_stream stream) {
  if (!f || !dev_K || !dev_X || !dev_G || !dev_Lambda || nrhs < 1 || nrhs > f->nrhs_max || ld < f->plan->p.N)
    return D3M_ERR_ARG;
  if (!f->factored || stale(f) || f->plan->p.nelim > 0) return D3M_ERR_STATE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  d3m_status st = solve_impl(f, dev_K, dev_G, dev_Lambda, nrhs, ld, s);
  if (st) return st;
  if (dev_dK)
    HIPCHK(launch_dk(dev_Lambda, dev_X, ld, nrhs, dev_dK, f->uv(), f->at<DkTaskDev>(f->lay.dkt),
                     (int)f->tab.dkt.size(), f->opt.dk_stored, s));
  f->last = s;
  return D3M_OK;
}

d3m_status d3m_reduce(d3m_factor f, const void* dev_A, const void* dev_F, int64_t ldf, void* dev_Kred,
                      void* dev_Gred, int64_t ldg, int32_t nrhs, d3m_stream stream) {
  if (!f || !dev_A || nrhs < 1 || nrhs > f->nrhs_max) return D3M_ERR_ARG;
  const PlanImpl& p = f->plan->p;
  if (p.nelim <= 0 || f->prec != 0) return D3M_ERR_STATE;  // needs a partial plan and a complex128 factor
  if (dev_F && (ldf < p.N || !dev_Gred || ldg < p.N - p.N_elim)) return D3M_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the eliminated blocks' factor, their Schur complement on the others
  HIPCHK(launch_prepare(f->at<int32_t>(f->lay.status), f->at<float>(f->lay.growth), p.nb, f->ctrl(), f->opt.tol,
                        f->opt.max_iter, s));
  HIPCHK(launch_scatter(dev_A, f->ws + f->lay.L, f->at<KPlaceDev>(f->lay.kp), (int)f->tab.kp.size(),
                        f->at<KPlaceDev>(f->lay.fills), (int)f->tab.fills.size(), f->at<double>(f->lay.kpart),
                        f->prec, s));
  d3m_status st = run_dag(f, 0, f->nrhs_max, nullptr, s);
  if (st != D3M_OK) return st;
  if (dev_Kred) {
    int maxe = 1;
    for (const auto& k : f->tab.kg) maxe = std::max(maxe, k.rows * k.cols);
    HIPCHK(launch_gather_red(f->ws + f->lay.L, dev_Kred, f->at<KPlaceDev>(f->lay.kg), (int)f->tab.kg.size(), p.nred,
                             maxe, s));
  }
  // the forward part of the solve: the reduced right-hand sides are left in
  // the rows of the blocks not eliminated (internal rows N_elim..N)
  if (dev_F) {
    HIPCHK(launch_perm_in(dev_F, ldf, f->ws + f->lay.W, 0, f->uv(), nrhs, nullptr, s));
    st = run_dag(f, 1, nrhs, nullptr, s);
    if (st != D3M_OK) return st;
    HIPCHK(launch_perm_rows(f->ws + f->lay.W, 0, dev_Gred, ldg, f->uv(), p.N_elim, p.N, nrhs, 1, s));
    f->red_nrhs = nrhs;
  } else {
    f->red_nrhs = 0;
  }
  f->last = s;
  f->factored = true;
  return D3M_OK;
}

d3m_status d3m_recover(d3m_factor f, const void* dev_Xred, int64_t ldx, void* dev_U, int64_t ldu, int32_t nrhs,
                       const void* dev_M, int64_t ldm, int32_t nports, void* dev_S, d3m_stream stream) {
  if (!f || !dev_Xred || !dev_U || nrhs < 1) return D3M_ERR_ARG;
  const PlanImpl& p = f->plan->p;
  if (p.nelim <= 0 || !f->factored || f->red_nrhs != nrhs) return D3M_ERR_STATE;  // after d3m_reduce with F
  if (ldx < p.N - p.N_elim || ldu < p.N || (nports > 0 && (!dev_M || !dev_S || ldm < p.N)) || nports < 0)
    return D3M_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the given solution of the blocks left into their rows, then the backward
  // part of the solve over the eliminated blocks
  HIPCHK(launch_perm_rows(dev_Xred, ldx, f->ws + f->lay.W, 0, f->uv(), p.N_elim, p.N, nrhs, 0, s));
  d3m_status st = run_dag(f, 2, nrhs, nullptr, s);
  if (st != D3M_OK) return st;
  HIPCHK(launch_perm_out(f->ws + f->lay.W, dev_U, ldu, f->uv(), nrhs, s));
  if (nports > 0) HIPCHK(launch_ports(dev_M, ldm, dev_U, ldu, p.N, nports, nrhs, dev_S, s));
  f->red_nrhs = 0;  // the forward part's z is used up
  f->last = s;
  return D3M_OK;
}

d3m_status d3m_status_sync(d3m_factor f, d3m_run_info* out) {
  if (!f || !out) return D3M_ERR_ARG;
  if (stale(f)) return D3M_ERR_STATE;
  HIPCHK(hipStreamSynchronize(f->last));
  std::memset(out, 0, sizeof(*out));
  int32_t st[3];
  IrCtrl c;
  int32_t flags[2];
  HIPCHK(hipMemcpy(st, f->at<int32_t>(f->lay.status), 12, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(&c, f->ctrl(), sizeof(c), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(flags, f->at<int32_t>(f->lay.flags), 8, hipMemcpyDeviceToHost));
  out->pivot_row = -1;
  out->status = D3M_OK;
  if (st[0] != 0x7fffffff) {
    int64_t q = st[0];
    if (f->opt.pivot) {
      // st[0] is a position inside a pivoted tile: the unknown there is the
      // tile's ipiv[q]-th
      const PlanImpl& p = f->plan->p;
      int32_t ip = 0;
      HIPCHK(hipMemcpy(&ip, f->at<int32_t>(f->lay.ipiv) + q, 4, hipMemcpyDeviceToHost));
      for (const Tile& T : p.tiles) {
        const int64_t t0 = p.panels[T.panel].prow0 + T.r0;
        if (q >= t0 && q < t0 + T.sz) { q = t0 + ip; break; }
      }
    }
    out->pivot_row = f->tab.perm[q];
    out->status = D3M_ZERO_PIVOT;
  }
  out->ir_iters = c.iters;
  out->fallbacks = st[2];
  out->knorm = c.knorm;
  out->eta = -1;
  for (int k = 0; k < 32; ++k) {
    out->eta_hist[k] = c.eta_hist[k];
    if (c.eta_hist[k] >= 0) out->eta = c.eta_hist[k];
  }
  if (out->status == D3M_OK && c.status) out->status = c.status;
  out->hang = flags[1];
  if (flags[1]) out->status = D3M_ERR_HANG;
  for (int w = 0; w < 2; ++w) {
    double tot = 0;
    for (int i = 0; i < f->nev[w]; ++i) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, f->ev[w][2 * i], f->ev[w][2 * i + 1]));
      tot += ms;
    }
    if (w == 0) { out->t_factor_dag_ms = tot; out->n_factor_dag = f->nev[0]; }
    else { out->t_solve_dag_ms = tot; out->n_solve_dag = f->nev[1]; }
    f->nev[w] = 0;
  }
  return (d3m_status)out->status;
}

d3m_status d3m_factor_block(d3m_factor f, int32_t J, int32_t I, void* host_out) {
  if (!f || !host_out) return D3M_ERR_ARG;
  if (stale(f)) return D3M_ERR_STATE;
  const PlanImpl& p = f->plan->p;
  if (I < 0 || I >= p.nb || J < 0 || J >= p.nb) return D3M_ERR_ARG;
  HIPCHK(hipStreamSynchronize(f->last));
  const Panel& P = p.panels[p.pos[I]];
  int rowoff = -1;
  for (int b = 0; b < P.npb; ++b)
    if (p.pblocks[P.pb0 + b].J == p.pos[J]) rowoff = p.pblocks[P.pb0 + b].prow;
  if (rowoff < 0) return D3M_ERR_ARG;
  const int nJ = p.n[J], nI = p.n[I];
  const size_t es = f->prec == 0 ? 16 : 8;
  std::vector<char> panel((size_t)P.H * nI * es);
  HIPCHK(hipMemcpy(panel.data(), f->ws + f->lay.L + P.off * es, panel.size(), hipMemcpyDeviceToHost));
  double* o = static_cast<double*>(host_out);
  for (int c = 0; c < nI; ++c)
    for (int r = 0; r < nJ; ++r) {
      size_t e = (size_t)(rowoff + r) + (size_t)c * P.H;
      double re, im;
      if (es == 16) {
        re = reinterpret_cast<double*>(panel.data())[2 * e];
        im = reinterpret_cast<double*>(panel.data())[2 * e + 1];
      } else {
        re = reinterpret_cast<float*>(panel.data())[2 * e];
        im = reinterpret_cast<float*>(panel.data())[2 * e + 1];
      }
      if (J == I && r < c) re = im = 0;  // upper part of the diagonal block is not part of the factor
      o[2 * ((size_t)r + (size_t)c * nJ)] = re;
      o[2 * ((size_t)r + (size_t)c * nJ) + 1] = im;
    }
  return D3M_OK;
}

d3m_status d3m_factor_pivots(d3m_factor f, int32_t I, int32_t* perm, void* doff_host) {
  if (!f || !perm || !doff_host) return D3M_ERR_ARG;
  const PlanImpl& p = f->plan->p;
  if (I < 0 || I >= p.nb) return D3M_ERR_ARG;
  if (!f->opt.pivot || !f->factored || stale(f)) return D3M_ERR_STATE;
  HIPCHK(hipStreamSynchronize(f->last));
  const Panel& P = p.panels[p.pos[I]];
  const size_t es = f->prec == 0 ? 16 : 8;
  std::vector<int32_t> ip(P.n);
  std::vector<char> dof((size_t)P.n * es);
  HIPCHK(hipMemcpy(ip.data(), f->at<int32_t>(f->lay.ipiv) + P.prow0, P.n * sizeof(int32_t), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(dof.data(), f->ws + f->lay.Doff + (size_t)P.prow0 * es, dof.size(), hipMemcpyDeviceToHost));
  double* o = static_cast<double*>(doff_host);
  for (int c = 0; c < P.nt; ++c) {
    const Tile& T = p.tiles[P.tile0 + c];
    for (int i = 0; i < T.sz; ++i) perm[T.r0 + i] = T.r0 + ip[T.r0 + i];
  }
  for (int i = 0; i < P.n; ++i) {
    if (es == 16) {
      o[2 * i] = reinterpret_cast<double*>(dof.data())[2 * i];
      o[2 * i + 1] = reinterpret_cast<double*>(dof.data())[2 * i + 1];
    } else {
      o[2 * i] = reinterpret_cast<float*>(dof.data())[2 * i];
      o[2 * i + 1] = reinterpret_cast<float*>(dof.data())[2 * i + 1];
    }
  }
  return D3M_OK;
}

d3m_status d3m_factor_set_trace(d3m_factor f, void* dev_buf, size_t bytes) {
  if (!f) return D3M_ERR_ARG;
  f->trace = dev_buf;
  f->trace_bytes = dev_buf ? bytes : 0;
  return D3M_OK;
}

d3m_status d3m_factor_tasks(d3m_factor f, int32_t solve, int32_t* kinds, int32_t* panels, int32_t* mnk, int32_t* count) {
  if (!f || !count) return D3M_ERR_ARG;
  const TaskDag& dag = solve ? f->plan->p.sdag : f->plan->p.fdag;
  const int n = (int)dag.tasks.size();
  if (kinds && panels && mnk)
    for (int i = 0; i < n; ++i) {
            kinds[i] = dag.tasks[i].kind & 0xff;
      panels[i] = dag.tasks[i].panel;
      mnk[3 * i] = dag.tasks[i].m;
      mnk[3 * i + 1] = dag.tasks[i].n;
      mnk[3 * i + 2] = dag.tasks[i].k;
    }
  *count = n;
  return D3M_OK;
}

void d3m_factor_destroy(d3m_factor f) {
  if (!f) return;
  for (int w = 0; w < 2; ++w)
    for (auto& e : f->ev[w]) (void)hipEventDestroy(e);
  delete f;
}

d3m_status d3m_debug_gemm(d3m_precision prec, int32_t m, int32_t n, int32_t k, int32_t amode, int32_t i0,
                          const void* A, int64_t lda, const void* d, const void* B, int64_t ldb, void* C,
                          int64_t ldc, double alpha, double beta, d3m_stream stream) {
  if (m < 1 || n < 1 || k < 0 || m > kTileMax || n > kTileMax || amode < 0 || amode > 2 || !A || !B || !C)
    return D3M_ERR_ARG;
  if (amode == 0 && lda < m) return D3M_ERR_ARG;
  if (amode == 1 && lda < k) return D3M_ERR_ARG;
  if (amode == 2 && (lda < k || i0 < 0 || i0 + m > lda)) return D3M_ERR_ARG;
  if (ldb < n || ldc < m) return D3M_ERR_ARG;
  HIPCHK(launch_debug_gemm(prec == D3M_C128 ? 0 : 1, m, n, k, amode, i0, A, lda, d, B, ldb, C, ldc, alpha, beta,
                           static_cast<hipStream_t>(stream)));
  return D3M_OK;
}

d3m_status d3m_tune_gemm(d3m_precision prec, void* dev_scratch, size_t bytes, int32_t* best_id, double* gflops_out,
                         int32_t* ncand) {
  if (!dev_scratch || !best_id || !ncand) return D3M_ERR_ARG;
  const int p = prec == D3M_C128 ? 0 : 1;
  const size_t es = p == 0 ? 16 : 8;
  const size_t need = (size_t)256 * 3 * 128 * 512 * es;
  if (bytes < need) return D3M_ERR_WORKSPACE;
  const int reps = 20;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipMemset(dev_scratch, 0, need));
  double rate[kBenchCands];
  for (int v = 0; v < kBenchCands; ++v) {
    HIPCHK(launch_gemm_bench(p, dev_scratch, 2, v, nullptr));
    HIPCHK(hipEventRecord(e0, nullptr));
    HIPCHK(launch_gemm_bench(p, dev_scratch, reps, v, nullptr));
    HIPCHK(hipEventRecord(e1, nullptr));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    const double per = v <= 1 ? 8.0 * 128 * 128 * 512 : 8.0 * 64 * 64 * 448;
    rate[v] = 256.0 * reps * per / (ms * 1e-3) / 1e9;
    if (gflops_out) gflops_out[v] = rate[v];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *best_id = rate[1] > rate[0] ? 1 : 0;
  *ncand = kBenchCands;
  return D3M_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batching
namespace {
struct BatchLayout {
  size_t ftasks, fsucc, fcnt, stasks, ssucc, scnt, counters, flags, iv, ctrls, bir, total;
};
BatchLayout batch_layout(const TaskDag& fd, const TaskDag& sd, int n) {
  BatchLayout l;
  size_t o = 0;
  // 64 bytes of slack after every section: a paired complex64 load of an
  // odd last row reads one element past its operand
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + std::max<size_t>(bytes, 1) + 64); return at; };
  l.ftasks = take(fd.tasks.size() * sizeof(Task));
  l.fsucc = take(fd.succ.size() * 4);
  l.fcnt = take(fd.npred.size() * 4);
  l.stasks = take(sd.tasks.size() * sizeof(Task));
  l.ssucc = take(sd.succ.size() * 4);
  l.scnt = take(sd.npred.size() * 4);
  l.counters = take(std::max(fd.tasks.size(), sd.tasks.size()) * 4);
  l.flags = take(4 * 4);
  l.iv = take(n * sizeof(InstView));
  l.ctrls = take(n * sizeof(IrCtrl*));
  l.bir = take(n * sizeof(BatchIrDev));
  l.total = o;
  return l;
}
}  // namespace

struct d3m_batch_s {
  std::vector<d3m_factor_s*> f;
  TaskDag fd, sd;
  BatchLayout lay{};
  char* ws = nullptr;
  int prec = 0;
  int nworkers = 256;
  int maxnrt = 1, maxnrhs = 1, minnrhs = 1 << 30, maxkng = 0;
  int totnb = 0, maxpanel = 1;  // scatter blocks of all instances, largest panel count of an instance
  int64_t maxtot = 1;  // largest N * nrhs of an instance
  template <typename P> P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
};

namespace {
d3m_status batch_dag(d3m_batch_s* b, bool solve, const int32_t* skip, hipStream_t s) {
  const TaskDag& dag = solve ? b->sd : b->fd;
  DagArgs a;
  a.tasks = b->at<Task>(solve ? b->lay.stasks : b->lay.ftasks);
  a.succ = b->at<int32_t>(solve ? b->lay.ssucc : b->lay.fsucc);
  a.counters = b->at<int32_t>(b->lay.counters);
  int32_t* flags = b->at<int32_t>(b->lay.flags);
  a.head = flags;
  a.abort_flag = flags + 1;
  a.skip = skip;
  a.inst = b->at<InstView>(b->lay.iv);
    a.ntask = (int32_t)dag.tasks.size();
  a.nrhs = 0;
  a.rhs_groups = 1;
  a.spin_limit_ns = 20LL * 1000 * 1000 * 1000;
  a.trace = nullptr;
  HIPCHK(launch_reset(a.counters, b->at<int32_t>(solve ? b->lay.scnt : b->lay.fcnt), a.ntask, a.head, a.abort_flag,
                      skip, s));
  HIPCHK(launch_dag(a, b->prec, b->nworkers, solve, s));
  return D3M_OK;
}
}  // namespace

extern "C" {

d3m_status d3m_batch_workspace_bytes(int32_t ninst, const d3m_factor* f, size_t* bytes) {
  if (ninst < 1 || !f || !bytes) return D3M_ERR_ARG;
  std::vector<const TaskDag*> fds, sds;
  for (int i = 0; i < ninst; ++i) {
    if (!f[i]) return D3M_ERR_ARG;
    fds.push_back(&f[i]->plan->p.fdag);
    sds.push_back(&f[i]->plan->p.sdag);
  }
  TaskDag fd = merge_dags(fds, 256), sd = merge_dags(sds, 256);
  *bytes = batch_layout(fd, sd, ninst).total;
  return D3M_OK;
}

d3m_status d3m_batch_create(int32_t ninst, const d3m_factor* f, void* dev_ws, size_t bytes, d3m_batch* out) {
  if (ninst < 1 || !f || !dev_ws || !out) return D3M_ERR_ARG;
  *out = nullptr;
  if (reinterpret_cast<uintptr_t>(dev_ws) % kAlign) return D3M_ERR_WORKSPACE;
  d3m_batch_s* b = new (std::nothrow) d3m_batch_s;
  if (!b) return D3M_ERR_ARG;
  std::vector<const TaskDag*> fds, sds;
  for (int i = 0; i < ninst; ++i) {
    if (!f[i] || f[i]->prec != f[0]->prec) { delete b; return D3M_ERR_ARG; }
    if (stale(f[i])) { delete b; return D3M_ERR_STATE; }
    b->f.push_back(f[i]);
    fds.push_back(&f[i]->plan->p.fdag);
    sds.push_back(&f[i]->plan->p.sdag);
  }
  b->prec = f[0]->prec;
  b->nworkers = device_cus();
  b->fd = merge_dags(fds, b->nworkers);
  b->sd = merge_dags(sds, b->nworkers);
  b->lay = batch_layout(b->fd, b->sd, ninst);
  if (bytes < b->lay.total) { delete b; return D3M_ERR_WORKSPACE; }
  b->ws = static_cast<char*>(dev_ws);
  std::vector<InstView> ivs(ninst);
  std::vector<IrCtrl*> ctrls(ninst);
  std::vector<BatchIrDev> bir(ninst);
  for (int i = 0; i < ninst; ++i) {
    if (hipMemcpy(&ivs[i], f[i]->ws + f[i]->lay.iv, sizeof(InstView), hipMemcpyDeviceToHost) != hipSuccess) {
      delete b;
      return D3M_ERR_HIP;
    }
    ctrls[i] = f[i]->ctrl();
    d3m_factor_s* fi = f[i];
    BatchIrDev& t = bir[i];
    std::memset(&t, 0, sizeof(t));
    t.W = fi->ws + fi->lay.W;
    t.X64 = fi->at<double2>(fi->lay.X64);
    t.R64 = fi->at<double2>(fi->lay.R64);
    t.P64 = fi->at<double2>(fi->lay.P64);
    t.rmax = fi->rmax();
    t.xmax = fi->xmax();
    t.bmax = fi->bmax();
    t.ctrl = fi->ctrl();
    t.uv = fi->uv();
    t.rt = fi->at<RTaskDev>(fi->lay.rt);
    t.nrt = (int32_t)fi->tab.rt.size();
    t.nrhs = fi->nrhs_max;
    t.tol = fi->opt.tol;
    t.max_iter = fi->opt.max_iter;
    t.L = fi->ws + fi->lay.L;
    t.kp = fi->at<KPlaceDev>(fi->lay.kp);
    t.fills = fi->at<KPlaceDev>(fi->lay.fills);
    t.part = fi->at<double>(fi->lay.kpart);
    t.kn = fi->kn();
    t.nkp = (int32_t)fi->tab.kp.size();
    t.nfill = (int32_t)fi->tab.fills.size();
    t.status = fi->at<int32_t>(fi->lay.status);
    t.growth = fi->at<float>(fi->lay.growth);
    t.flag = fi->at<int32_t>(fi->lay.flags) + 1;
    t.npanel = fi->plan->p.nb;
    t.sb0 = b->totnb;
    b->totnb += t.nkp + t.nfill;
    b->maxpanel = std::max(b->maxpanel, (int)t.npanel);
    b->maxnrt = std::max(b->maxnrt, (int)t.nrt);
    b->maxkng = std::max(b->maxkng, (int)t.kn.ngroups);
    b->maxnrhs = std::max(b->maxnrhs, (int)t.nrhs);
    b->minnrhs = std::min(b->minnrhs, (int)t.nrhs);
    b->maxtot = std::max<int64_t>(b->maxtot, fi->plan->p.N * t.nrhs);
  }
  auto up = [&](size_t off, const void* src, size_t n) {
    return n == 0 || hipMemcpy(b->ws + off, src, n, hipMemcpyHostToDevice) == hipSuccess;
  };
  bool ok = up(b->lay.ftasks, b->fd.tasks.data(), b->fd.tasks.size() * sizeof(Task)) &&
            up(b->lay.fsucc, b->fd.succ.data(), b->fd.succ.size() * 4) &&
            up(b->lay.fcnt, b->fd.npred.data(), b->fd.npred.size() * 4) &&
            up(b->lay.stasks, b->sd.tasks.data(), b->sd.tasks.size() * sizeof(Task)) &&
            up(b->lay.ssucc, b->sd.succ.data(), b->sd.succ.size() * 4) &&
            up(b->lay.scnt, b->sd.npred.data(), b->sd.npred.size() * 4) &&
            up(b->lay.iv, ivs.data(), ivs.size() * sizeof(InstView)) &&
            up(b->lay.ctrls, ctrls.data(), ctrls.size() * sizeof(IrCtrl*)) &&
            up(b->lay.bir, bir.data(), bir.size() * sizeof(BatchIrDev));
  if (!ok) { delete b; return D3M_ERR_HIP; }
  *out = b;
  return D3M_OK;
}

d3m_status d3m_batch_run(d3m_batch b, const void* const* K, const void* const* B, void* const* X,
                         const int32_t* nrhs, const int64_t* ld, d3m_stream stream) {
  if (!b || !K || !B || !X || !nrhs || !ld) return D3M_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = (int)b->f.size();
  for (int i = 0; i < n; ++i) {
    const d3m_factor_s* f = b->f[i];
    if (!K[i] || !B[i] || !X[i] || nrhs[i] != f->nrhs_max || ld[i] < f->plan->p.N) return D3M_ERR_ARG;
    if (stale(f)) return D3M_ERR_STATE;
  }
  // the user's pointers into the instance table, then state reset,
  // scatter/convert and ||K|| of all instances (a launch each) and one
  // persistent factor launch
  BatchIrDev* tab = b->at<BatchIrDev>(b->lay.bir);
  HIPCHK(launch_batch_user(tab, n, K, B, X, ld, s));
  HIPCHK(launch_batch_setup(tab, n, b->prec, b->totnb, b->maxkng, b->maxpanel, s));
  d3m_status st = batch_dag(b, false, nullptr, s);
  if (st) return st;
  HIPCHK(launch_batch_flags(tab, n, b->at<int32_t>(b->lay.flags) + 1, s));
  // the refinement bookkeeping of all instances: one launch per kind and step
  HIPCHK(launch_batch_begin(tab, n, b->prec, b->maxtot, s));
  st = batch_dag(b, true, nullptr, s);
  if (st) return st;
  int32_t* allstop = b->at<int32_t>(b->lay.flags) + 2;
  const int max_iter = b->f[0]->opt.max_iter;
  if (b->prec == 1) HIPCHK(launch_batch_cvt_up(tab, n, b->maxtot, s));
  for (int it = 0; it <= (b->prec == 1 ? max_iter : 0); ++it) {
    HIPCHK(launch_batch_check(tab, n, b->prec, b->maxnrt, b->minnrhs, b->maxnrhs, b->maxtot,
                              b->prec == 0 ? 2 : (it == max_iter ? 1 : 0), s));
    if (b->prec == 1 && it < max_iter) HIPCHK(launch_batch_cvt_down(tab, n, b->maxtot, s));
    if (b->prec == 0 || it == max_iter) break;
    HIPCHK(launch_all_stop(b->at<IrCtrl*>(b->lay.ctrls), n, allstop, s));
    st = batch_dag(b, true, allstop, s);
    if (st) return st;
    HIPCHK(launch_batch_axpy_up(tab, n, b->maxtot, s));
  }
  HIPCHK(launch_batch_perm_out(tab, n, b->prec, b->maxtot, s));
  for (int i = 0; i < n; ++i) {
    b->f[i]->last = s;
    b->f[i]->factored = true;
  }
  return D3M_OK;
}

void d3m_batch_destroy(d3m_batch b) { delete b; }

}  // extern "C"
