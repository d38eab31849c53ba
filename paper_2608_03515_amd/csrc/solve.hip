// Solve phase of the host runtime: the V-cycle (paper's two-level scheme applied recursively)
// and the batched, right-preconditioned FGMRES(m) driver (paper: FGMRES outer solver to a
// relative residual of 1e-10).
//
// A batch is a workspace of `cap` right-hand-side slots on one stream.  Every kernel runs over
// all slots and skips those whose device state is inactive, so slots can be admitted at any
// restart-cycle boundary while the others keep iterating (the server admits requests this
// way), and a right-hand side's arithmetic does not depend on the other slots.  The host
// reads the per-slot state once per cycle through a pinned mirror and an event; it never
// blocks inside a batch, so several batches on several streams are driven from one thread.
#include <algorithm>
#include <cstring>

#include "runtime.hpp"

namespace amamg {
namespace rt {

// Blocks per right-hand side of the Gram-Schmidt and norm kernels: about 4096 blocks in all
// (16 per compute unit), at least 8 elements per thread once that many blocks exist (the
// per-block reduction of the previous pass's partials is then amortised), at most one block
// per 256 elements and at most kMaxKrylovBlocks.
static int krylov_blocks(int64_t n, int nrhs) {
  const int64_t want = std::max<int64_t>(n / 2048, (4096 + nrhs - 1) / nrhs);
  return int(std::max<int64_t>(1, std::min<int64_t>({int64_t(kMaxKrylovBlocks), n / 256, want})));
}

// ------------------------------------------------------------------------------ workspace

Workspace::~Workspace() { release(); }

void Workspace::release() {
  if (graph) (void)hipGraphExecDestroy(graph);
  graph = nullptr;
  graph_key.clear();
  if (block) (void)hipFree(block);
  if (hst) (void)hipHostFree(hst);
  if (hst2) (void)hipHostFree(hst2);
  if (hadmit) (void)hipHostFree(hadmit);
  if (hhist) (void)hipHostFree(hhist);
  if (ev) (void)hipEventDestroy(ev);
  block = nullptr;
  block_bytes = 0;
  hst = hst2 = nullptr;
  hadmit = nullptr;
  hhist = nullptr;
  host_cap = host_hist = 0;
  ev = nullptr;
  lv.clear();
  shape.clear();
  cap = m = hist_cap = 0;
}

// complex entries per right-hand side of the coarsest GMRES basis (0 for the exact solve)
static size_t coarsest_basis(const amamg_hierarchy* h) {
  if (!(h->prm.coarsest_tol > 0)) return 0;
  return size_t(h->prm.coarsest_max_iters + 1) * size_t(h->lv.back().g.ndof());
}

static size_t level_rpart_count(const LevelData& L, Real prec) {
  return size_t(L.g.nI) * L.g.nJ * restrict_chunks(L.g, L.nf, prec) * L.g.ncol();
}

size_t workspace_bytes(const amamg_hierarchy* h, int cap, int m, Real prec, int hist_cap) {
  const int64_t n = h->lv[0].g.ndof();
  const size_t rs = prec == F64 ? sizeof(double2) : sizeof(float2);
  size_t b = sizeof(double2) * size_t(m + 1) * cap * n + size_t(m) * cap * n * rs +
             sizeof(double2) * size_t(cap) * n + sizeof(double2) * size_t(cap) * (3 * (m + 1) * m / 2 + 4 * m) +
             sizeof(double2) * size_t(3) * cap * kMaxKrylovBlocks * 32 + sizeof(double2) * size_t(cap) * hist_cap +
             sizeof(double2) * size_t(cap) * 64 + sizeof(double) * size_t(cap) * m + 2 * 256;
  for (size_t k = 1; k < h->lv.size(); ++k) b += 3 * size_t(cap) * h->lv[k].g.ndof() * rs;
  b += size_t(cap) * n * rs;
  for (size_t k = 0; k + 1 < h->lv.size(); ++k) b += size_t(cap) * level_rpart_count(h->lv[k], prec) * rs;
  b += sizeof(double2) * size_t(cap) * coarsest_basis(h) + 256;
  return b;
}

static std::vector<int64_t> shape_of(const amamg_hierarchy* h, Real prec) {
  std::vector<int64_t> s;
  for (size_t k = 0; k < h->lv.size(); ++k) {
    s.push_back(h->lv[k].g.ndof());
    s.push_back(k + 1 < h->lv.size() ? int64_t(level_rpart_count(h->lv[k], prec)) : 0);
  }
  s.push_back(int64_t(coarsest_basis(h)));
  return s;
}

bool workspace_fits(const Workspace& ws, const amamg_hierarchy* h, int cap, int m, Real prec, int hist_cap) {
  return ws.cap == cap && ws.m == m && ws.prec == prec && ws.hist_cap >= hist_cap &&
         ws.shape == shape_of(h, prec);
}

// Device layout of a workspace; `take` hands out 256-byte aligned ranges of the block.
template <typename Take>
static void layout(Workspace& ws, const amamg_hierarchy* h, int cap, int m, Real prec, int hist_cap, Take take) {
  const int64_t n = h->lv[0].g.ndof();
  const size_t rs = prec == F64 ? sizeof(double2) : sizeof(float2);
  ws.V = (double2*)take(sizeof(double2) * size_t(m + 1) * cap * n);
  ws.Z = take(size_t(m) * cap * n * rs);
  ws.w = (double2*)take(sizeof(double2) * size_t(cap) * n);
  ws.H = (double2*)take(sizeof(double2) * size_t(cap) * (m + 1) * m);
  ws.g = (double2*)take(sizeof(double2) * size_t(cap) * (m + 1));
  ws.cs = (double*)take(sizeof(double) * size_t(cap) * m);
  ws.sn = (double2*)take(sizeof(double2) * size_t(cap) * m);
  ws.y = (double2*)take(sizeof(double2) * size_t(cap) * m);
  ws.part = (double2*)take(sizeof(double2) * size_t(3) * cap * kMaxKrylovBlocks * 32);
  ws.coef = (double2*)take(sizeof(double2) * size_t(cap) * 64);
  ws.zsc = (double*)take(sizeof(double) * size_t(cap) * m);
  ws.st = (RhsState*)take(sizeof(RhsState) * cap);
  ws.st2 = (RhsState*)take(sizeof(RhsState) * cap);
  ws.admit = (int*)take(sizeof(int) * cap);
  ws.hist = (double2*)take(sizeof(double2) * size_t(cap) * hist_cap);
  ws.lv.assign(h->lv.size(), Workspace::Lev{});
  for (size_t k = 1; k < h->lv.size(); ++k) {
    const int64_t nd = h->lv[k].g.ndof();
    ws.lv[k].f = take(size_t(cap) * nd * rs);
    ws.lv[k].x = take(size_t(cap) * nd * rs);
    ws.lv[k].tmp = take(size_t(cap) * nd * rs);
  }
  ws.lv[0].tmp = take(size_t(cap) * n * rs);
  for (size_t k = 0; k + 1 < h->lv.size(); ++k)
    ws.lv[k].rpart = take(size_t(cap) * level_rpart_count(h->lv[k], prec) * rs);
  if (coarsest_basis(h) > 0) ws.lv.back().kry = (double2*)take(sizeof(double2) * size_t(cap) * coarsest_basis(h));
}

void ensure_workspace(Workspace& ws, const amamg_hierarchy* h, int cap, int m, Real prec, int hist_cap) {
  if (workspace_fits(ws, h, cap, m, prec, hist_cap)) return;
  size_t off = 0;
  char* base = nullptr;
  auto take = [&](size_t bytes) -> void* {
    off = (off + 255) & ~size_t(255);
    void* p = base ? base + off : nullptr;
    off += std::max<size_t>(bytes, 1);
    return p;
  };
  layout(ws, h, cap, m, prec, hist_cap, take);      // sizes only
  if (ws.block_bytes < off) {
    if (ws.block) (void)hipFree(ws.block);
    ws.block = nullptr;
    ws.block_bytes = 0;
    HIPCHECK(hipMalloc(&ws.block, off));
    ws.block_bytes = off;
  }
  base = static_cast<char*>(ws.block);
  off = 0;
  layout(ws, h, cap, m, prec, hist_cap, take);
  if (ws.host_cap < cap) {
    if (ws.hst) (void)hipHostFree(ws.hst);
    if (ws.hst2) (void)hipHostFree(ws.hst2);
    if (ws.hadmit) (void)hipHostFree(ws.hadmit);
    ws.hst = ws.hst2 = nullptr;
    ws.hadmit = nullptr;
    ws.host_cap = 0;
    HIPCHECK(hipHostMalloc((void**)&ws.hst, sizeof(RhsState) * cap, hipHostMallocDefault));
    HIPCHECK(hipHostMalloc((void**)&ws.hst2, sizeof(RhsState) * cap, hipHostMallocDefault));
    HIPCHECK(hipHostMalloc((void**)&ws.hadmit, sizeof(int) * cap, hipHostMallocDefault));
    ws.host_cap = cap;
  }
  if (size_t(ws.host_hist) < size_t(cap) * hist_cap) {
    if (ws.hhist) (void)hipHostFree(ws.hhist);
    ws.hhist = nullptr;
    ws.host_hist = 0;
    HIPCHECK(hipHostMalloc((void**)&ws.hhist, sizeof(double2) * size_t(cap) * hist_cap, hipHostMallocDefault));
    ws.host_hist = cap * hist_cap;
  }
  if (!ws.ev) HIPCHECK(hipEventCreateWithFlags(&ws.ev, hipEventDisableTiming));
  // every slot starts free (inactive, done)
  std::memset(ws.hst, 0, sizeof(RhsState) * cap);
  for (int r = 0; r < cap; ++r) ws.hst[r].done = 1;
  HIPCHECK(hipMemcpy(ws.st, ws.hst, sizeof(RhsState) * cap, hipMemcpyHostToDevice));
  ws.cap = cap;
  ws.m = m;
  ws.prec = prec;
  ws.hist_cap = hist_cap;
  ws.shape = shape_of(h, prec);
}

// ------------------------------------------------------------------------------ V-cycle

struct SolveCtx {
  amamg_hierarchy* h;
  Workspace* ws;
  hipStream_t s;
  Real T;
  LinkStore smooth_links, mat_links;
  int nrhs;        // slots (grid extent of every launch)
  int step;        // Arnoldi step of the current V-cycle (kernel timer)
  int group;       // kernel-timer group
  int fine_tc;     // launch shapes chosen by the tuner (0 = default)
  const int* gs_rb;
};

// x = M_k f (V-cycle of the paper's two-level scheme, recursively; start x = 0)
static void vcycle(const SolveCtx& c, int k, Real fprec, const void* f, void* x) {
  amamg_hierarchy* h = c.h;
  LevelData& L = h->lv[k];
  Workspace::Lev& WL = c.ws->lv[k];
  const Geom& g = L.g;
  const int64_t nd = g.ndof();
  const RhsState* st = c.ws->st;
  const bool f64 = c.T == F64;
  if (L.coarsest) {
    if (h->prm.coarsest_tol > 0)
      coarsest_gmres(c.s, c.T, L.Acm, f, x, int(nd), c.nrhs, nd, st, h->prm.coarsest_tol,
                     h->prm.coarsest_max_iters, WL.kry);
    else
      dense_apply(c.s, c.T, L.Ainv, f, x, int(nd), c.nrhs, nd, st);
    return;
  }
  LevelData& C = h->lv[k + 1];
  Workspace::Lev& WC = c.ws->lv[k + 1];
  const int64_t ndc = C.g.ndof();
  const void* P = f64 ? (const void*)L.P : (const void*)L.P32;
  const int pre = h->prm.pre_sweeps, post = h->prm.post_sweeps;
  amamg_gauge* gg = h->gauge;
  amamg_context* ctx = gg->ctx;
  const void* U0 = link0(gg, c.smooth_links);
  const void* U1 = link1(gg, c.smooth_links);
  const void* Ak = f64 ? (const void*)L.A : (const void*)L.A32;
  const void* Dk = f64 ? (const void*)L.Dinv : (const void*)L.Dinv32;
  const double cb = f64 ? 16.0 : 8.0;   // bytes per complex value
  if (pre > 0) {
    HIPCHECK(hipMemsetAsync(x, 0, nd * c.nrhs * (f64 ? 16 : 8), c.s));
    for (int sw = 0; sw < pre; ++sw) {
      if (k == 0)
        for (int col = 0; col < 2; ++col)
          wilson_gs(c.s, c.smooth_links, U0, U1, c.T, x, (const double2*)f, g.Lt, g.Lx, h->m0, col, c.nrhs, nd, st);
      else
        for (int col = 0; col < 16; ++col)
          stencil_gs(c.s, c.T, Ak, Dk, x, f, g.Lt, g.Lx, g.b, coarse_colour(col), c.nrhs, nd, st);
    }
    if (k == 0)
      wilson_apply(c.s, c.smooth_links, U0, U1, c.T, x, c.T, WL.tmp, (const double2*)f, g.Lt, g.Lx, h->m0, c.nrhs, nd, st);
    else
      stencil_apply(c.s, c.T, Ak, x, WL.tmp, f, g.Lt, g.Lx, g.b, c.nrhs, nd, st);
    restrict_(c.s, c.T, P, L.rows, L.nrows, L.nf, c.T, WL.tmp, WC.f, WL.rpart, g, c.nrhs, nd, ndc, st);
  } else {
    // per rhs: the fine vector in, the coarse vector out; per launch: the owned rows' weights
    const double fb = fprec == F64 ? 16 : 8;
    const double owned = double(nd) * (1.0 - double(g.o * g.o) / double(g.a * g.a));
    const int rec = k == 0 ? timer_start(ctx, c.s, AMAMG_KT_RESTRICT0, c.step, c.group,
                                         double(nd) * fb + double(ndc) * cb, owned * g.ncol() * cb)
                           : -1;
    restrict_(c.s, c.T, P, L.rows, L.nrows, L.nf, fprec, f, WC.f, WL.rpart, g, c.nrhs, nd, ndc, st);
    timer_stop(ctx, c.s, rec);
  }
  vcycle(c, k + 1, c.T, WC.f, WC.x);
  // fine level without pre-smoothing: the post-sweeps run fused, from the prolongated
  // correction in the level's scratch vector into x
  const bool fused = k == 0 && pre == 0 && (post == 1 || post == 2);
  {
    const double owned = double(nd) * (1.0 - double(g.o * g.o) / double(g.a * g.a));
    // per rhs: the coarse vector in, the fine vector out; per launch: the owned rows' weights
    const int rec = k == 0 ? timer_start(ctx, c.s, AMAMG_KT_PROLONG0, c.step, c.group,
                                         double(nd) * cb + double(ndc) * cb, owned * g.ncol() * cb)
                           : -1;
    prolong(c.s, c.T, P, L.rows, L.nrows, L.nf, WC.x, fused ? WL.tmp : x, g, pre > 0 ? 1 : 0, c.nrhs, nd,
            ndc, st);
    timer_stop(ctx, c.s, rec);
  }
  if (fused) {
    // per rhs: the prolongated correction in, x out, b (FP64) in; per launch: the links
    const double cl = c.smooth_links == LINK_F64 ? 16 : c.smooth_links == LINK_F32 ? 8 : 4;
    const int rec = timer_start(ctx, c.s, AMAMG_KT_FINE_GS, c.step, c.group,
                                double(g.nnode()) * (2 * 2 * cb + 32), double(g.nnode()) * 2 * cl);
    wilson_gs_sweeps(c.s, c.smooth_links, U0, U1, c.T, WL.tmp, x, (const double2*)f, g.Lt, g.Lx, h->m0, post,
                     c.nrhs, nd, st, c.fine_tc);
    timer_stop(ctx, c.s, rec);
    return;
  }
  for (int sw = 0; sw < post; ++sw) {
    if (k == 0) {
      const double cl = c.smooth_links == LINK_F64 ? 16 : c.smooth_links == LINK_F32 ? 8 : 4;
      for (int col = 0; col < 2; ++col) {
        const int rec = timer_start(ctx, c.s, AMAMG_KT_FINE_GS, c.step, c.group,
                                    double(g.nnode()) * (2 * cb + 16), double(g.nnode()) * 2 * cl);
        wilson_gs(c.s, c.smooth_links, U0, U1, c.T, x, (const double2*)f, g.Lt, g.Lx, h->m0, col, c.nrhs, nd, st);
        timer_stop(ctx, c.s, rec);
      }
    } else {
      // the four colour blocks of the sweep order (four colours each)
      for (int qb = 0; qb < 4; ++qb) {
        // per rhs: x of the whole level in, f in and x out at the block's four colours; per
        // launch: those nodes' 25 stencil blocks and diagonal-block inverses
        const double ncn = double(g.nnode()) / 16.0;
        const int rec = k == 1 ? timer_start(ctx, c.s, AMAMG_KT_COARSE_GS, c.step, c.group,
                                             4.0 * 2.0 * ncn * g.b * cb + double(nd) * cb,
                                             4.0 * ncn * 26.0 * g.b * g.b * cb)
                               : -1;
        stencil_gs_block(c.s, c.T, Ak, Dk, x, f, g.Lt, g.Lx, g.b, qb, c.nrhs, nd, st, c.gs_rb ? c.gs_rb[k] : 0,
                         h->prm.block_smoother);
        timer_stop(ctx, c.s, rec);
      }
    }
  }
}

// --------------------------------------------------------------------------------- batch

static void check_solve_params(const amamg_solve_params& p) {
  REQUIRE(p.restart >= 1 && p.restart <= 31, AMAMG_ERR_INVALID_ARG, "restart must be in [1, 31]");
  REQUIRE(p.max_iters >= 1, AMAMG_ERR_INVALID_ARG, "max_iters must be >= 1");
  REQUIRE(p.rel_tol > 0 && std::isfinite(p.rel_tol), AMAMG_ERR_INVALID_ARG, "rel_tol must be > 0");
  REQUIRE(p.precision >= 0 && p.precision <= 2, AMAMG_ERR_INVALID_ARG, "unknown precision");
  REQUIRE(p.groups >= 0 && p.groups <= 16, AMAMG_ERR_INVALID_ARG, "groups must be in [0, 16]");
}

static SolveCtx make_ctx(const Batch& bt) {
  SolveCtx c{bt.h, bt.ws, bt.s, bt.p.precision == AMAMG_FP64 ? F64 : F32, LINK_F64, LINK_F64,
             bt.ws->cap, 0, bt.group, bt.fine_tc, bt.gs_rb.empty() ? nullptr : bt.gs_rb.data()};
  if (bt.p.precision == AMAMG_MIXED_FP32) { c.smooth_links = LINK_F32; c.mat_links = LINK_F32; }
  if (bt.p.precision == AMAMG_MIXED_FP32_BF16LINKS) { c.smooth_links = LINK_BF16; c.mat_links = LINK_F32; }
  return c;
}

static KrylovDims dims(const Batch& bt) {
  const int64_t n = bt.h->lv[0].g.ndof();
  return KrylovDims{n, bt.ws->cap, krylov_blocks(n, bt.ws->cap), bt.p.restart};
}

// ------------------------------------------------------------------------------ autotuning

// Mean time in microseconds of `run` on stream s (one untimed run, then the timed ones).
template <typename F> static double time_us(hipStream_t s, F run) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  // ten timed runs: candidates a microsecond or two apart per launch (the level-1 sweeps of a
  // single right-hand side) are told apart reliably
  constexpr int kReps = 10;
  run();
  HIPCHECK(hipEventRecord(e0, s));
  for (int q = 0; q < kReps; ++q) run();
  HIPCHECK(hipEventRecord(e1, s));
  HIPCHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return double(ms) * 1000.0 / kReps;
}

// The tuned value for `key`: cached, or (mode AUTO) the fastest candidate by `measure`, or
// (mode FORCE) candidate `force`, or (mode OFF) 0 = the kernel's default.
template <typename F>
static int tuned(Tuner& t, const std::array<int, 6>& key, const std::vector<int>& cand, F measure) {
  std::lock_guard<std::mutex> lk(t.mu);
  if (t.mode == AMAMG_TUNE_OFF) return 0;
  if (t.mode == AMAMG_TUNE_FORCE) return cand[std::min<size_t>(std::max(t.force, 0), cand.size() - 1)];
  auto it = t.entries.find(key);
  if (it != t.entries.end()) return it->second.choice;
  Tuner::Entry e;
  e.cand = cand;
  for (int v : cand) e.us.push_back(measure(v));
  e.choice = cand[std::min_element(e.us.begin(), e.us.end()) - e.us.begin()];
  t.entries[key] = e;
  return e.choice;
}

// Launch shapes of this batch's smoothers.  Runs before any right-hand side is admitted: the
// candidates are timed on the workspace's own vectors, zeroed, which hold nothing yet.
static void tune_batch(Batch& bt) {
  amamg_hierarchy* h = bt.h;
  Workspace* ws = bt.ws;
  amamg_context* ctx = h->gauge->ctx;
  const SolveCtx c = make_ctx(bt);
  const int prec = int(bt.p.precision), cap = ws->cap;
  const size_t rs = c.T == F64 ? sizeof(double2) : sizeof(float2);
  bt.fine_tc = 0;
  bt.gs_rb.assign(h->lv.size(), 0);
  amamg_gauge* gg = h->gauge;
  const Geom& g0 = h->lv[0].g;
  if (h->lv.size() > 1 && h->prm.pre_sweeps == 0 && (h->prm.post_sweeps == 1 || h->prm.post_sweeps == 2)) {
    std::vector<int> cand = {16};
    if (g0.Lx >= 32) cand.push_back(32);
    if (g0.Lx >= 64 && c.T == F32) cand.push_back(64);
    const int64_t nd = g0.ndof();
    void* xin = ws->lv[0].tmp;
    void* xo = ws->Z;
    const double2* b = ws->V;
    bt.fine_tc = tuned(ctx->tuner, {Tuner::FINE_GS_TILE, g0.Lt, g0.Lx, g0.b, prec, cap}, cand, [&](int tc) {
      HIPCHECK(hipMemsetAsync(xin, 0, rs * cap * nd, bt.s));
      HIPCHECK(hipMemsetAsync(xo, 0, rs * cap * nd, bt.s));
      HIPCHECK(hipMemsetAsync(ws->V, 0, sizeof(double2) * cap * nd, bt.s));
      return time_us(bt.s, [&] {
        wilson_gs_sweeps(bt.s, c.smooth_links, link0(gg, c.smooth_links), link1(gg, c.smooth_links), c.T, xin, xo,
                         b, g0.Lt, g0.Lx, h->m0, h->prm.post_sweeps, cap, nd, nullptr, tc);
      });
    });
  }
  for (size_t k = 1; k + 1 < h->lv.size(); ++k) {
    const Geom& g = h->lv[k].g;
    if (g.b != 8) continue;
    const bool f32 = c.T == F32;
    std::vector<int> cand;
    if (f32 && gs_on_matrix_cores(g.Lt, g.Lx, h->prm.block_smoother)) {
      cand = {8, 12, 24};                   // offsets per load batch of the matrix-core sweep
    } else {
      // > 0: colour-pair launches with that many rhs per wave (FP64: 0 = the generic pair
      // kernel); < 0: one launch per colour block (kGsNodeWaves: one wave per node)
      if (f32 && cap < 2) continue;
      cand = f32 ? std::vector<int>{1} : std::vector<int>{0};
      if (cap >= 2) cand.push_back(2);
      if (cap >= 4) cand.push_back(4);
      cand.push_back(-1);
      if (cap >= 2) cand.push_back(-2);
      cand.push_back(kGsNodeWaves);
    }
    const int64_t nd = g.ndof();
    Workspace::Lev& WL = ws->lv[k];
    const void* Ak = f32 ? (const void*)h->lv[k].A32 : (const void*)h->lv[k].A;
    const void* Dk = f32 ? (const void*)h->lv[k].Dinv32 : (const void*)h->lv[k].Dinv;
    bt.gs_rb[k] = tuned(ctx->tuner, {Tuner::COARSE_GS_RHS, g.Lt, g.Lx, g.b, prec, cap}, cand, [&](int rb) {
      HIPCHECK(hipMemsetAsync(WL.x, 0, rs * cap * nd, bt.s));
      HIPCHECK(hipMemsetAsync(WL.f, 0, rs * cap * nd, bt.s));
      return time_us(bt.s, [&] {
        for (int qb = 0; qb < 4; ++qb)
          stencil_gs_block(bt.s, c.T, Ak, Dk, WL.x, WL.f, g.Lt, g.Lx, g.b, qb, cap, nd, nullptr, rb,
                           h->prm.block_smoother);
      });
    });
  }
  check_launch();
}

void Batch::init(amamg_hierarchy* h_, Workspace* ws_, hipStream_t s_, const amamg_solve_params& p_,
                 const double2* b_, double2* x_, int group_) {
  h = h_; ws = ws_; s = s_; p = p_; b = b_; x = x_; group = group_;
  REQUIRE(workspace_fits(*ws, h, ws->cap, p.restart, p.precision == AMAMG_FP64 ? F64 : F32, 2 * p.max_iters + 2),
          AMAMG_ERR_INVALID_ARG, "workspace does not match the hierarchy and solve parameters");
  cycle_in.assign(ws->cap, 0);
  pending.clear();
  cycle_enqueued = false;
  const SolveCtx c = make_ctx(*this);
  ensure_links(h->gauge, c.smooth_links);
  ensure_links(h->gauge, c.mat_links);
  // the links' copies are made on the context stream
  if (s != h->gauge->ctx->stream) {
    HIPCHECK(hipEventRecord(ws->ev, h->gauge->ctx->stream));
    HIPCHECK(hipStreamWaitEvent(s, ws->ev, 0));
  }
  tune_batch(*this);
}

void Batch::admit_begin(const std::vector<int>& slots) {
  const KrylovDims kd = dims(*this);
  std::memset(ws->hst2, 0, sizeof(RhsState) * ws->cap);
  for (int r = 0; r < ws->cap; ++r) ws->hadmit[r] = 0;
  for (int r : slots) {
    ws->hst2[r].active = 1;
    ws->hadmit[r] = 1;
  }
  pending = slots;
  HIPCHECK(hipMemcpyAsync(ws->st2, ws->hst2, sizeof(RhsState) * ws->cap, hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(ws->admit, ws->hadmit, sizeof(int) * ws->cap, hipMemcpyHostToDevice, s));
  // ||b|| and fresh states of the admitted slots; non-finite input is refused before x is touched
  norm_control(s, kd, b, ws->part, ws->st2, 1, ws->g, p.rel_tol, p.max_iters, ws->hist, ws->hist_cap);
  check_launch();
  HIPCHECK(hipMemcpyAsync(ws->hst2, ws->st2, sizeof(RhsState) * ws->cap, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipEventRecord(ws->ev, s));
}

std::vector<int> Batch::admit_nonfinite() const {
  std::vector<int> out;
  for (int r : pending)
    if (ws->hst2[r].nonfinite) out.push_back(r);
  return out;
}

void Batch::admit_finish(const std::vector<int>& reject, bool use_initial_guess) {
  const KrylovDims kd = dims(*this);
  const int64_t n = kd.n;
  bool any = false;
  for (int r : pending) {
    if (std::find(reject.begin(), reject.end(), r) != reject.end()) {
      ws->hst2[r].active = 0;     // excluded: the slot stays free
      ws->hadmit[r] = 0;
      continue;
    }
    any = true;
    if (!use_initial_guess) HIPCHECK(hipMemsetAsync(x + int64_t(r) * n, 0, sizeof(double2) * n, s));
  }
  pending.clear();
  if (!any) return;
  if (!reject.empty()) {
    HIPCHECK(hipMemcpyAsync(ws->st2, ws->hst2, sizeof(RhsState) * ws->cap, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(ws->admit, ws->hadmit, sizeof(int) * ws->cap, hipMemcpyHostToDevice, s));
  }
  amamg_gauge* gg = h->gauge;
  // r = b - D x into V_0, its norm, the first cycle start, V_0 = r / ||r||
  wilson_apply(s, LINK_F64, gg->U, gg->U + int64_t(gg->nt) * gg->nx, F64, x, F64, ws->V, b, gg->nt, gg->nx,
               h->m0, ws->cap, n, ws->st2);
  norm_control(s, kd, ws->V, ws->part, ws->st2, 2, ws->g, p.rel_tol, p.max_iters, ws->hist, ws->hist_cap);
  scale_next(s, kd, ws->V, ws->V, ws->st2);
  merge_states(s, ws->st, ws->st2, ws->admit, ws->cap);
  check_launch();
}

void Batch::enqueue_state_read() {
  HIPCHECK(hipMemcpyAsync(ws->hst, ws->st, sizeof(RhsState) * ws->cap, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipEventRecord(ws->ev, s));
}

bool Batch::ready() const {
  const hipError_t e = hipEventQuery(ws->ev);
  if (e == hipSuccess) return true;
  if (e == hipErrorNotReady) return false;
  throw Fail{AMAMG_ERR_DEVICE, std::string("hipEventQuery: ") + hipGetErrorString(e)};
}

// After a synchronisation: account the pending launches of this group; served(step) = rhs
// active at that step.
template <typename F> static void timer_flush(amamg_context* ctx, int group, F served) {
  KernelTimer& t = ctx->timer;
  size_t keep = 0;
  for (size_t i = 0; i < t.pending.size(); ++i) {
    const auto r = t.pending[i];
    if (r.group != group) {
      t.pending[keep++] = r;
      continue;
    }
    const int n = served(r.step);
    if (n <= 0) continue;
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, t.events[r.e0], t.events[r.e1]));
    t.launches[r.family] += 1;
    t.total_ms[r.family] += ms;
    t.total_bytes[r.family] += r.bytes_per_rhs * n + r.bytes_per_launch;
  }
  t.pending.resize(keep);
}

bool Batch::cycle_boundary() {
  amamg_context* ctx = h->gauge->ctx;
  if (cycle_enqueued)
    timer_flush(ctx, group, [&](int step) {
      int cnt = 0;
      for (int r = 0; r < ws->cap; ++r) cnt += (cycle_in[r] && ws->hst[r].last_k > step) ? 1 : 0;
      return cnt;
    });
  cycle_enqueued = false;
  bool any = false;
  for (int r = 0; r < ws->cap; ++r) {
    cycle_in[r] = ws->hst[r].in_cycle;
    any = any || ws->hst[r].in_cycle;
  }
  return any;
}

// Everything a captured cycle bakes in: buffer addresses, launch shapes, the stream and the
// values passed by value (mass, tolerances, tuned choices), and the hierarchy's setup count.
static std::vector<uint64_t> graph_key(const Batch& bt) {
  uint64_t tol;
  std::memcpy(&tol, &bt.p.rel_tol, sizeof tol);
  uint64_t m0;
  std::memcpy(&m0, &bt.h->m0, sizeof m0);
  std::vector<uint64_t> k{uint64_t(uintptr_t(bt.h)), bt.h->generation, m0, uint64_t(uintptr_t(bt.s)),
                          uint64_t(uintptr_t(bt.b)), uint64_t(uintptr_t(bt.x)),
                          uint64_t(uintptr_t(bt.ws->block)), uint64_t(bt.ws->cap),
                          uint64_t(bt.ws->hist_cap), uint64_t(uint32_t(bt.p.precision)),
                          uint64_t(uint32_t(bt.p.restart)), uint64_t(uint32_t(bt.p.max_iters)), tol,
                          uint64_t(uint32_t(bt.group)), uint64_t(uint32_t(bt.fine_tc))};
  for (int v : bt.gs_rb) k.push_back(uint64_t(uint32_t(v)));
  const amamg_gauge* gg = bt.h->gauge;
  const Workspace& w = *bt.ws;
  for (const void* q : {(const void*)gg->U, (const void*)gg->U32, (const void*)gg->U16, (const void*)w.V,
                        (const void*)w.Z, (const void*)w.st, (const void*)w.part, (const void*)w.coef,
                        (const void*)w.hist})
    k.push_back(uint64_t(uintptr_t(q)));
  for (const Workspace::Lev& l : w.lv)
    for (const void* q : {l.f, l.x, l.tmp, l.rpart, (void*)l.kry}) k.push_back(uint64_t(uintptr_t(q)));
  return k;
}

void Batch::enqueue_cycle() {
  // (the legacy null stream cannot be captured; the kernel timer and pre-smoothing record
  // event and memset nodes, which stay out of graphs)
  const bool use_graph = p.graphs != 0 && s != nullptr && h->gauge->ctx->timer.mask == 0 &&
                         h->prm.pre_sweeps == 0;
  if (!use_graph) {
    enqueue_cycle_kernels();
    return;
  }
  std::vector<uint64_t> key = graph_key(*this);
  if (!ws->graph || key != ws->graph_key) {
    if (ws->graph) (void)hipGraphExecDestroy(ws->graph);
    ws->graph = nullptr;
    ws->graph_key.clear();
    HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    try {
      enqueue_cycle_kernels();
    } catch (...) {
      (void)hipStreamEndCapture(s, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHECK(hipStreamEndCapture(s, &g));
    const hipError_t e = hipGraphInstantiate(&ws->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      ws->graph = nullptr;
      throw Fail{AMAMG_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
    }
    ws->graph_key = std::move(key);
  }
  HIPCHECK(hipGraphLaunch(ws->graph, s));
  cycle_enqueued = true;
}

void Batch::enqueue_cycle_kernels() {
  for (int j = 0; j < p.restart; ++j) {
    enqueue_step_front(j);
    enqueue_step_krylov(j);
  }
  enqueue_cycle_tail();
}

// Arnoldi step j up to w = D z_j: the V-cycle z_j = M u_j and the matvec.
void Batch::enqueue_step_front(int j) {
  SolveCtx c = make_ctx(*this);
  const KrylovDims kd = dims(*this);
  const int64_t n = kd.n, vsj = int64_t(ws->cap) * n;
  const Real T = c.T;
  const size_t zs = T == F64 ? sizeof(double2) : sizeof(float2);
  amamg_gauge* gg = h->gauge;
  amamg_context* ctx = gg->ctx;
  const int nt = gg->nt, nx = gg->nx;
  const void* Um0 = link0(gg, c.mat_links);
  const void* Um1 = link1(gg, c.mat_links);
  const double cl = c.mat_links == LINK_F64 ? 16 : 8;
  // Timer steps: served(step) counts the rhs whose cycle reached more than `step` columns.
  // The V-cycle, matvec and Gram pass of step j run for every rhs still active at step j
  // (> j - 1 columns); the update runs for those that go on after column j - 1 (> j).
  double2* uj = ws->V + j * vsj;
  void* zj = (char*)ws->Z + size_t(j) * vsj * zs;
  c.step = j - 1;
  vcycle(c, 0, F64, uj, zj);
  const int rec = timer_start(ctx, s, AMAMG_KT_FINE_MATVEC, j - 1, group, double(nt) * nx * (2 * zs + 32),
                              double(nt) * nx * 2 * cl);
  wilson_apply(s, c.mat_links, Um0, Um1, T, zj, F64, ws->w, nullptr, nt, nx, h->m0, ws->cap, n, ws->st);
  timer_stop(ctx, s, rec);
}

// Arnoldi step j's Gram-Schmidt: pass A (slots 0..j and w), control, pass B.
void Batch::enqueue_step_krylov(int j) {
  const KrylovDims kd = dims(*this);
  const int64_t n = kd.n, vsj = int64_t(ws->cap) * n;
  amamg_context* ctx = h->gauge->ctx;
  const double inner_tol = p.precision == AMAMG_FP64 ? 0.0 : 1e-5;
  RhsState* st = ws->st;
  double2* p1 = ws->part;
  // family DOTS = the Gram passes (slots 0..j and w), family UPDATE = the updates (read slots
  // 0..j and w; write slot j + 1 and, for j > 0, slot j)
  int rec = timer_start(ctx, s, AMAMG_KT_DOTS, j - 1, group, double(j + 2) * n * 16);
  gram(s, kd, ws->V, vsj, j + 1, ws->w, p1, st);
  timer_stop(ctx, s, rec);
  lag_control(s, kd, p1, st, ws->H, ws->cs, ws->sn, ws->g, ws->coef, ws->zsc, j, 1, p.rel_tol, inner_tol,
              p.max_iters, ws->hist, ws->hist_cap);
  rec = timer_start(ctx, s, AMAMG_KT_UPDATE, j, group, double(j + (j > 0 ? 4 : 3)) * n * 16);
  lag_update(s, kd, ws->V, vsj, j + 1, ws->w, ws->coef, st, j > 0);
  timer_stop(ctx, s, rec);
  check_launch();
}

// End of a cycle: the last column, the solution update, the true residual and the next
// cycle's start.
void Batch::enqueue_cycle_tail() {
  const KrylovDims kd = dims(*this);
  const int64_t n = kd.n, vsj = int64_t(ws->cap) * n;
  const int m = p.restart;
  const Real T = p.precision == AMAMG_FP64 ? F64 : F32;
  amamg_gauge* gg = h->gauge;
  amamg_context* ctx = gg->ctx;
  const int nt = gg->nt, nx = gg->nx;
  const double inner_tol = T == F64 ? 0.0 : 1e-5;
  RhsState* st = ws->st;
  double2* p1 = ws->part;
  // the rhs that ran all m steps: last column from the reorthogonalisation of slot m
  int rec = timer_start(ctx, s, AMAMG_KT_DOTS, m - 1, group, double(m + 1) * n * 16);
  gram(s, kd, ws->V, vsj, m + 1, nullptr, p1, st);
  timer_stop(ctx, s, rec);
  lag_control(s, kd, p1, st, ws->H, ws->cs, ws->sn, ws->g, ws->coef, ws->zsc, m, 0, p.rel_tol, inner_tol,
              p.max_iters, ws->hist, ws->hist_cap);
  backsolve_update(s, kd, st, ws->H, ws->g, ws->zsc, ws->y, T, ws->Z, vsj, x);
  wilson_apply(s, LINK_F64, gg->U, gg->U + int64_t(nt) * nx, F64, x, F64, ws->V, b, nt, nx, h->m0, ws->cap, n, st);
  norm_control(s, kd, ws->V, p1, st, 3, ws->g, p.rel_tol, p.max_iters, ws->hist, ws->hist_cap);
  scale_next(s, kd, ws->V, ws->V, st);
  check_launch();
  cycle_enqueued = true;
}

// This batch as a segment of the multi-batch Krylov launches.
KrylovSeg Batch::krylov_seg() const {
  KrylovSeg q{};
  q.dm = dims(*this);
  q.V = ws->V;
  q.vsj = int64_t(ws->cap) * q.dm.n;
  q.w = ws->w;
  q.part = ws->part;
  q.st = ws->st;
  q.coef = ws->coef;
  q.zsc = ws->zsc;
  q.aa = ArnoldiArgs{ws->H, ws->cs, ws->sn, ws->g, 0, p.rel_tol, p.precision == AMAMG_FP64 ? 0.0 : 1e-5,
                     p.max_iters, ws->hist, ws->hist_cap};
  return q;
}

std::vector<double2> Batch::history(int slot) const {
  const int len = std::min(ws->hst[slot].hist_len, ws->hist_cap);
  std::vector<double2> out(len);
  if (len > 0) {
    HIPCHECK(hipMemcpyAsync(out.data(), ws->hist + int64_t(slot) * ws->hist_cap, sizeof(double2) * len,
                            hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
  }
  return out;
}

// --------------------------------------------------------------------------- plain solve

// Drive the batches until every one has finished; blocks on the oldest outstanding event
// when no batch can advance.
amamg_status run_solve(amamg_hierarchy* h, int nrhs, const double2* b, double2* x,
                       const amamg_solve_params& p, amamg_solve_info* info) {
  REQUIRE(nrhs >= 1, AMAMG_ERR_INVALID_ARG, "nrhs must be >= 1");
  check_solve_params(p);
  amamg_context* ctx = h->gauge->ctx;
  const int G = std::max(1, std::min(p.groups, nrhs));
  const int64_t n = h->lv[0].g.ndof();
  const Real T = p.precision == AMAMG_FP64 ? F64 : F32;
  const int hist_cap = 2 * p.max_iters + 2;
  while (int(h->ws.size()) < G) h->ws.push_back(new Workspace());
  while (int(h->streams.size()) < G - 1) {
    hipStream_t sx;
    HIPCHECK(hipStreamCreateWithFlags(&sx, hipStreamNonBlocking));
    h->streams.push_back(sx);
  }
  // group g: right-hand sides [off[g], off[g + 1])
  std::vector<int> off(G + 1, 0);
  for (int g = 0; g < G; ++g) off[g + 1] = off[g] + nrhs / G + (g < nrhs % G ? 1 : 0);
  std::vector<Batch> bt(G);
  ctx->timer.pending.clear();
  for (int g = 0; g < G; ++g) {
    const int q = off[g + 1] - off[g];
    Workspace& ws = *h->ws[g];
    // reused only at exactly this slot count (the reduction blocking depends on it) and shape
    ensure_workspace(ws, h, q, p.restart, T, hist_cap);
  }
  for (int g = 0; g < G; ++g) {
    hipStream_t s = g == 0 ? ctx->stream : h->streams[g - 1];
    bt[g].init(h, h->ws[g], s, p, b + int64_t(off[g]) * n, x + int64_t(off[g]) * n, g);
  }
  // phase 1: input check of every group; a non-finite right-hand side fails the whole call
  // before any x is written
  std::vector<int> all;
  for (int g = 0; g < G; ++g) {
    all.resize(off[g + 1] - off[g]);
    for (size_t r = 0; r < all.size(); ++r) all[r] = int(r);
    bt[g].admit_begin(all);
  }
  try {
    for (int g = 0; g < G; ++g) HIPCHECK(hipEventSynchronize(h->ws[g]->ev));
    for (int g = 0; g < G; ++g) {
      const std::vector<int> bad = bt[g].admit_nonfinite();
      REQUIRE(bad.empty(), AMAMG_ERR_NONFINITE,
              "non-finite value in right-hand side " + std::to_string(off[g] + (bad.empty() ? 0 : bad[0])));
    }
    for (int g = 0; g < G; ++g) {
      bt[g].admit_finish({}, p.use_initial_guess != 0);
      bt[g].enqueue_state_read();
    }
    // phase 2: restart cycles, each batch advanced as soon as its last state read has landed
    std::vector<int> done(G, 0);
    std::vector<uint64_t> stamp(G, 0);
    uint64_t clock = 0;
    int left = G;
    while (left > 0) {
      bool progressed = false;
      for (int g = 0; g < G; ++g) {
        if (done[g] || !bt[g].ready()) continue;
        progressed = true;
        if (!bt[g].cycle_boundary()) {
          done[g] = 1;
          --left;
          continue;
        }
        bt[g].enqueue_cycle();
        bt[g].enqueue_state_read();
        stamp[g] = ++clock;
      }
      if (!progressed) {
        int oldest = -1;
        for (int g = 0; g < G; ++g)
          if (!done[g] && (oldest < 0 || stamp[g] < stamp[oldest])) oldest = g;
        HIPCHECK(hipEventSynchronize(h->ws[oldest]->ev));
      }
    }
  } catch (...) {
    for (int g = 0; g < G; ++g) (void)hipStreamSynchronize(bt[g].s);
    throw;
  }
  // results
  h->history.assign(nrhs, {});
  bool all_conv = true, nonfinite = false;
  for (int g = 0; g < G; ++g) {
    Workspace& ws = *h->ws[g];
    const int q = off[g + 1] - off[g];
    HIPCHECK(hipMemcpyAsync(ws.hhist, ws.hist, sizeof(double2) * size_t(q) * ws.hist_cap, hipMemcpyDeviceToHost, bt[g].s));
    HIPCHECK(hipStreamSynchronize(bt[g].s));
    for (int r = 0; r < q; ++r) {
      const RhsState& s = ws.hst[r];
      const double2* hh = ws.hhist + size_t(r) * ws.hist_cap;
      h->history[off[g] + r].assign(hh, hh + std::min(s.hist_len, ws.hist_cap));
      all_conv = all_conv && s.converged;
      nonfinite = nonfinite || s.nonfinite;
      if (info) {
        amamg_solve_info& o = info[off[g] + r];
        o.iterations = s.iters;
        o.restarts = s.restarts;
        o.converged = s.converged;
        o.reserved = 0;
        o.true_rel_residual = s.true_res;
      }
    }
  }
  REQUIRE(!nonfinite, AMAMG_ERR_NONFINITE, "non-finite value during the solve");
  return all_conv ? AMAMG_OK : AMAMG_NOT_CONVERGED;
}

// ------------------------------------------------------------------------ several lattices

// Several hierarchies (lattices of any sizes) solved together: one batch per lattice on one of
// up to four streams, advanced in lock step.  Step j runs every lattice's V-cycle and matvec on
// its own stream, then one launch of each Gram-Schmidt kernel for all lattices (KrylovSeg
// segments, persistent workgroups over the lattices' work items), then the next step; a cycle
// ends with each lattice's own tail.  With p.graphs a whole round (all lattices' cycles, with
// the stream fork and join) is captured into one HIP graph and launched once per round; the
// graph is captured again when the set of lattices still iterating changes.  Each right-hand
// side gets bitwise its result in a plain solve of its lattice with the same batch size.
amamg_status run_solve_multi(const std::vector<amamg_hierarchy*>& hs, const std::vector<int>& nrhs,
                             const std::vector<const double2*>& b, const std::vector<double2*>& x,
                             const amamg_solve_params& p, amamg_solve_info* info, hipStream_t root) {
  check_solve_params(p);
  const int L = int(hs.size());
  REQUIRE(L >= 1 && int(nrhs.size()) == L, AMAMG_ERR_INVALID_ARG, "need at least one lattice");
  amamg_context* ctx = hs[0]->gauge->ctx;
  for (int l = 0; l < L; ++l) {
    REQUIRE(nrhs[l] >= 1, AMAMG_ERR_INVALID_ARG, "nrhs must be >= 1 for every lattice");
    REQUIRE(hs[l]->gauge->ctx == ctx, AMAMG_ERR_INVALID_ARG, "all hierarchies must share one context");
    for (int k = 0; k < l; ++k) REQUIRE(hs[k] != hs[l], AMAMG_ERR_INVALID_ARG, "a hierarchy is listed twice");
  }
  const Real T = p.precision == AMAMG_FP64 ? F64 : F32;
  const int hist_cap = 2 * p.max_iters + 2;
  const int NS = std::min(L, 4);
  std::vector<hipStream_t> ss(NS, nullptr);
  std::vector<hipEvent_t> evs(L + 1, nullptr);
  KrylovSeg* dseg = nullptr;
  hipGraphExec_t graph = nullptr;
  std::vector<Batch> bt(L);
  auto cleanup = [&] {
    for (hipStream_t sx : ss)
      if (sx) (void)hipStreamSynchronize(sx);
    if (root) (void)hipStreamSynchronize(root);
    if (graph) (void)hipGraphExecDestroy(graph);
    for (hipEvent_t e : evs)
      if (e) (void)hipEventDestroy(e);
    for (hipStream_t sx : ss)
      if (sx) (void)hipStreamDestroy(sx);
    if (dseg) (void)hipFree(dseg);
  };
  try {
    for (int q = 0; q < NS; ++q) HIPCHECK(hipStreamCreateWithFlags(&ss[q], hipStreamNonBlocking));
    for (hipEvent_t& e : evs) HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ctx->timer.pending.clear();
    for (int l = 0; l < L; ++l) {
      amamg_hierarchy* h = hs[l];
      if (h->ws.empty()) h->ws.push_back(new Workspace());
      ensure_workspace(*h->ws[0], h, nrhs[l], p.restart, T, hist_cap);
    }
    // every lattice's stream starts after the caller's queued work
    HIPCHECK(hipEventRecord(evs[L], root));
    for (int q = 0; q < NS; ++q) HIPCHECK(hipStreamWaitEvent(ss[q], evs[L], 0));
    // streams by longest-first greedy balance of each lattice's unknowns x right-hand sides, so
    // that the streams' shares of a lock step are about equal
    std::vector<int> order(L), sid(L, 0);
    for (int l = 0; l < L; ++l) order[l] = l;
    auto work = [&](int l) { return double(hs[l]->lv[0].g.ndof()) * nrhs[l]; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return work(a) > work(c); });
    std::vector<double> load(NS, 0.0);
    for (int l : order) {
      const int q = int(std::min_element(load.begin(), load.end()) - load.begin());
      sid[l] = q;
      load[q] += work(l);
    }
    for (int l = 0; l < L; ++l) bt[l].init(hs[l], hs[l]->ws[0], ss[sid[l]], p, b[l], x[l], l);
    // admission of every right-hand side, as a plain solve's
    for (int l = 0; l < L; ++l) {
      std::vector<int> all(nrhs[l]);
      for (int r = 0; r < nrhs[l]; ++r) all[r] = r;
      bt[l].admit_begin(all);
    }
    for (int l = 0; l < L; ++l) HIPCHECK(hipEventSynchronize(hs[l]->ws[0]->ev));
    for (int l = 0; l < L; ++l) {
      const std::vector<int> bad = bt[l].admit_nonfinite();
      REQUIRE(bad.empty(), AMAMG_ERR_NONFINITE, "non-finite value in a right-hand side of lattice " + std::to_string(l));
    }
    for (int l = 0; l < L; ++l) {
      bt[l].admit_finish({}, p.use_initial_guess != 0);
      bt[l].enqueue_state_read();
    }
    for (int l = 0; l < L; ++l) HIPCHECK(hipEventSynchronize(hs[l]->ws[0]->ev));
    // segments of the multi-lattice Krylov launches
    std::vector<KrylovSeg> seg(L);
    int blocks = 0, rhs = 0;
    for (int l = 0; l < L; ++l) {
      seg[l] = bt[l].krylov_seg();
      seg[l].item0 = blocks;
      seg[l].rhs0 = rhs;
      blocks += seg[l].dm.nrhs * seg[l].dm.nblk;
      rhs += seg[l].dm.nrhs;
    }
    HIPCHECK(hipMalloc(&dseg, sizeof(KrylovSeg) * L));
    HIPCHECK(hipMemcpy(dseg, seg.data(), sizeof(KrylovSeg) * L, hipMemcpyHostToDevice));
    const hipStream_t s0 = ss[0];
    // (the kernel timer records events and pre-smoothing a memset, which stay out of graphs)
    bool use_graph = p.graphs != 0 && ctx->timer.mask == 0;
    for (int l = 0; l < L; ++l) use_graph = use_graph && hs[l]->prm.pre_sweeps == 0;
    std::vector<char> live(L, 0), captured;
    for (;;) {
      bool any = false;
      for (int l = 0; l < L; ++l) {
        live[l] = bt[l].cycle_boundary() ? 1 : 0;
        any = any || live[l];
      }
      if (!any) break;
      // one round: the lattices' steps in lock step, then their tails
      auto enqueue_round = [&] {
        HIPCHECK(hipEventRecord(evs[L], s0));
        for (int q = 1; q < NS; ++q) HIPCHECK(hipStreamWaitEvent(ss[q], evs[L], 0));
        for (int j = 0; j < p.restart; ++j) {
          for (int l = 0; l < L; ++l)
            if (live[l]) bt[l].enqueue_step_front(j);
          for (int q = 1; q < NS; ++q) {
            HIPCHECK(hipEventRecord(evs[q], ss[q]));
            HIPCHECK(hipStreamWaitEvent(s0, evs[q], 0));
          }
          gram_multi(s0, dseg, L, blocks, j + 1);
          lag_control_multi(s0, dseg, L, rhs, j, 1);
          lag_update_multi(s0, dseg, L, blocks, j + 1, j > 0 ? 1 : 0);
          HIPCHECK(hipEventRecord(evs[0], s0));
          for (int q = 1; q < NS; ++q) HIPCHECK(hipStreamWaitEvent(ss[q], evs[0], 0));
        }
        for (int l = 0; l < L; ++l)
          if (live[l]) bt[l].enqueue_cycle_tail();
        for (int q = 1; q < NS; ++q) {
          HIPCHECK(hipEventRecord(evs[q], ss[q]));
          HIPCHECK(hipStreamWaitEvent(s0, evs[q], 0));
        }
        check_launch();
      };
      if (use_graph) {
        // a captured round stays in use while the lattices still iterating hold at least half
        // of its work: the finished ones' kernels find no active right-hand side and return
        double live_work = 0, cap_work = 0;
        for (int l = 0; l < L; ++l) {
          if (live[l]) live_work += work(l);
          if (!captured.empty() && captured[l]) cap_work += work(l);
        }
        bool covers = !captured.empty();
        for (int l = 0; l < L && covers; ++l) covers = !live[l] || captured[l];
        if (!graph || !covers || live_work < 0.5 * cap_work) {
          if (graph) (void)hipGraphExecDestroy(graph);
          graph = nullptr;
          HIPCHECK(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
          hipGraph_t g = nullptr;
          try {
            enqueue_round();
          } catch (...) {
            (void)hipStreamEndCapture(s0, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
          }
          HIPCHECK(hipStreamEndCapture(s0, &g));
          const hipError_t e = hipGraphInstantiate(&graph, g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
          if (e != hipSuccess) {
            graph = nullptr;
            throw Fail{AMAMG_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
          }
          captured = live;
        }
        HIPCHECK(hipGraphLaunch(graph, s0));
        for (int l = 0; l < L; ++l) live[l] = captured[l];   // their state reads follow the graph
      } else {
        enqueue_round();
      }
      // state reads on the lattices' streams after the round
      HIPCHECK(hipEventRecord(evs[L], s0));
      for (int q = 1; q < NS; ++q) HIPCHECK(hipStreamWaitEvent(ss[q], evs[L], 0));
      for (int l = 0; l < L; ++l) {
        bt[l].cycle_enqueued = live[l] != 0;
        bt[l].enqueue_state_read();
      }
      for (int l = 0; l < L; ++l) HIPCHECK(hipEventSynchronize(hs[l]->ws[0]->ev));
    }
  } catch (...) {
    cleanup();
    throw;
  }
  // the caller's stream follows the solve
  for (int q = 0; q < NS; ++q) {
    HIPCHECK(hipEventRecord(evs[q], ss[q]));
    HIPCHECK(hipStreamWaitEvent(root, evs[q], 0));
  }
  bool all_conv = true, nonfinite = false;
  int off = 0;
  for (int l = 0; l < L; ++l) {
    amamg_hierarchy* h = hs[l];
    Workspace& ws = *h->ws[0];
    HIPCHECK(hipMemcpyAsync(ws.hhist, ws.hist, sizeof(double2) * size_t(nrhs[l]) * ws.hist_cap, hipMemcpyDeviceToHost,
                            bt[l].s));
    HIPCHECK(hipStreamSynchronize(bt[l].s));
    h->history.assign(nrhs[l], {});
    for (int r = 0; r < nrhs[l]; ++r) {
      const RhsState& st = ws.hst[r];
      const double2* hh = ws.hhist + size_t(r) * ws.hist_cap;
      h->history[r].assign(hh, hh + std::min(st.hist_len, ws.hist_cap));
      all_conv = all_conv && st.converged;
      nonfinite = nonfinite || st.nonfinite;
      if (info) {
        amamg_solve_info& o = info[off + r];
        o.iterations = st.iters;
        o.restarts = st.restarts;
        o.converged = st.converged;
        o.reserved = 0;
        o.true_rel_residual = st.true_res;
      }
    }
    off += nrhs[l];
  }
  cleanup();
  REQUIRE(!nonfinite, AMAMG_ERR_NONFINITE, "non-finite value during the solve");
  return all_conv ? AMAMG_OK : AMAMG_NOT_CONVERGED;
}

}  // namespace rt
}  // namespace amamg

amamg_hierarchy::~amamg_hierarchy() {
  for (auto* w : ws) delete w;
  for (hipStream_t s : streams) (void)hipStreamDestroy(s);
}
