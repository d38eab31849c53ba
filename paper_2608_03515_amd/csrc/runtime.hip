// Host runtime and C ABI of the AM-AMG library: handles, the GPU setup pipeline and the entry
// points.  Every numerical step runs in the kernels of this directory; the host only sequences
// launches, owns device memory and reads per-rhs status once per restart cycle.
#include <atomic>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "runtime.hpp"

using namespace amamg;
using namespace amamg::rt;

namespace {

int period_of(int L) {
  for (int d = 5; d <= L; ++d)
    if (L % d == 0) return d;
  return L;
}

// Galerkin probing: probe columns per batch (the bc columns of nb node colours, at most 64
// columns when bc <= 64)
int probe_batch_colours(int bc, int ncolour) { return std::max(1, std::min(ncolour, 64 / bc)); }


}  // namespace

namespace amamg {

TimedLaunch& timed_launch() {
  thread_local TimedLaunch t;
  return t;
}

namespace rt {

amamg_status fail(amamg_context* ctx, const Fail& f) {
  if (ctx) ctx->err = f.msg;
  return f.code;
}

// Fields are moved one site (two spin components, 16 or 32 bytes) per vector access.
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Fail{AMAMG_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e)};
}

static int timer_event(KernelTimer& t, size_t idx) {
  while (t.events.size() <= idx) {
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    t.events.push_back(e);
  }
  return int(idx);
}

// Start / stop recording one launch of `family` at Arnoldi step `step` of batch `group`.
// Families launched by one kernel arm the launch hook (events stamped by the kernel itself);
// the fine restriction (two kernels) and the level-1 smoother's colour blocks (one or two
// kernels) are bracketed by stream events.
static bool bracketed(int family) { return family == AMAMG_KT_RESTRICT0 || family == AMAMG_KT_COARSE_GS; }
int timer_start(amamg_context* ctx, hipStream_t s, int family, int step, int group, double bytes_per_rhs,
                double bytes_per_launch) {
  KernelTimer& t = ctx->timer;
  if (!(t.mask & (1u << family))) return -1;
  // event pairs are reused once their records have been flushed
  size_t slot = 0;
  for (const auto& r : t.pending) slot = std::max(slot, size_t(r.e1) + 1);
  const int e0 = timer_event(t, slot), e1 = timer_event(t, slot + 1);
  if (bracketed(family)) HIPCHECK(hipEventRecord(t.events[e0], s));
  else timed_launch() = TimedLaunch{t.events[e0], t.events[e1]};
  t.pending.push_back({e0, e1, step, family, group, bytes_per_rhs, bytes_per_launch});
  return int(t.pending.size()) - 1;
}
void timer_stop(amamg_context* ctx, hipStream_t s, int rec) {
  if (rec < 0) return;
  KernelTimer& t = ctx->timer;
  const auto& r = t.pending[rec];
  TimedLaunch& tl = timed_launch();
  if (bracketed(r.family) || tl.start == t.events[r.e0]) {
    // bracketing events (or a hook no launch consumed: the record then spans nothing)
    if (tl.start == t.events[r.e0]) HIPCHECK(hipEventRecord(t.events[r.e0], s));
    HIPCHECK(hipEventRecord(t.events[r.e1], s));
  }
  tl = TimedLaunch{};
}

bool finite_all(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}


void ensure_links(amamg_gauge* gg, LinkStore ls) {
  hipStream_t s = gg->ctx->stream;
  const int64_t n = 2 * int64_t(gg->nt) * gg->nx;
  if (ls == LINK_F32 && gg->v32 != gg->version) {
    if (!gg->U32) gg->U32 = gg->mem.alloc<float2>(n);
    links_to_f32(s, gg->U, gg->U32, n);
    gg->v32 = gg->version;
  }
  if (ls == LINK_BF16 && gg->v16 != gg->version) {
    if (!gg->U16) gg->U16 = gg->mem.alloc<bf16c>(n);
    links_to_bf16(s, gg->U, gg->U16, n);
    gg->v16 = gg->version;
  }
}

const void* link0(amamg_gauge* g, LinkStore ls) {
  return ls == LINK_F64 ? (const void*)g->U : ls == LINK_F32 ? (const void*)g->U32 : (const void*)g->U16;
}
const void* link1(amamg_gauge* g, LinkStore ls) {
  const int64_t v = int64_t(g->nt) * g->nx;
  return ls == LINK_F64 ? (const void*)(g->U + v) : ls == LINK_F32 ? (const void*)(g->U32 + v)
                                                                      : (const void*)(g->U16 + v);
}


}  // namespace rt
}  // namespace amamg

namespace {

// footprint tables: postab[pos] = F index or -(1 + vcol); followed by fpos[nf]
std::vector<int> footprint_tables(int a, int o, int b, int* nf_out) {
  const int fpw = a + o, bc = o * o * b;
  std::vector<int> postab(fpw * fpw), fpos;
  for (int dt = 0; dt < fpw; ++dt)
    for (int dx = 0; dx < fpw; ++dx) {
      const int pos = dt * fpw + dx;
      const bool vt = dt < o || dt >= a, vx = dx < o || dx >= a;
      if (vt && vx) {
        const int ct = dt >= a, cx = dx >= a;
        const int pt = dt - ct * a, px = dx - cx * a;
        postab[pos] = -(1 + (2 * ct + cx) * bc + (pt * o + px) * b);
      } else {
        postab[pos] = int(fpos.size());
        fpos.push_back(pos);
      }
    }
  *nf_out = int(fpos.size());
  postab.insert(postab.end(), fpos.begin(), fpos.end());
  return postab;
}

struct LevelPlan {
  int Lt, Lx, b;
};

std::vector<LevelPlan> plan_levels(int nt, int nx, const amamg_setup_params& p) {
  REQUIRE(p.levels >= 2 && p.levels <= 8, AMAMG_ERR_INVALID_ARG, "levels must be in [2, 8]");
  REQUIRE(p.overlap >= 1 && p.overlap < p.agg_size, AMAMG_ERR_UNSUPPORTED_SHAPE,
          "overlap must satisfy 1 <= o < a");
  REQUIRE(p.norm >= 0 && p.norm <= 2, AMAMG_ERR_INVALID_ARG, "unknown normalisation");
  REQUIRE(p.norm != AMAMG_NORM_TESTVEC || (p.n_test_vectors >= 1 && p.n_test_vectors <= 16),
          AMAMG_ERR_INVALID_ARG, "n_test_vectors must be in [1, 16]");
  REQUIRE(p.test_vector_sweeps >= 0 && p.pre_sweeps >= 0 && p.post_sweeps >= 0,
          AMAMG_ERR_INVALID_ARG, "sweep counts must be >= 0");
  REQUIRE(std::isfinite(p.coarsest_tol) && p.coarsest_tol >= 0 && p.coarsest_tol < 1, AMAMG_ERR_INVALID_ARG,
          "coarsest_tol must be in [0, 1)");
  REQUIRE(p.coarsest_tol == 0 || (p.coarsest_max_iters >= 1 && p.coarsest_max_iters <= kCoarsestGmresMaxSteps),
          AMAMG_ERR_INVALID_ARG, "coarsest_max_iters must be in [1, 32]");
  REQUIRE(p.block_smoother >= 0 && p.block_smoother <= 2, AMAMG_ERR_INVALID_ARG, "block_smoother must be 0, 1 or 2");
  REQUIRE(p.aug_vectors >= 0 && (p.aug_vectors == 0 || (p.norm == AMAMG_NORM_TESTVEC &&
                                                        p.aug_vectors <= p.n_test_vectors)),
          AMAMG_ERR_INVALID_ARG, "aug_vectors needs the TESTVEC normalisation and at most n_test_vectors");
  std::vector<LevelPlan> out;
  int Lt = nt, Lx = nx, b = 2;
  const int a = p.agg_size, o = p.overlap;
  for (int k = 0; k < p.levels; ++k) {
    out.push_back({Lt, Lx, b});
    if (k == p.levels - 1) break;
    REQUIRE(Lt % a == 0 && Lx % a == 0 && Lt / a >= 2 && Lx / a >= 2, AMAMG_ERR_UNSUPPORTED_SHAPE,
            "aggregate size must divide every non-coarsest grid with at least 2 wirebaskets per direction");
    if (k >= 1) {
      REQUIRE(Lt % 4 == 0 && Lx % 4 == 0 && Lt >= 8 && Lx >= 8, AMAMG_ERR_UNSUPPORTED_SHAPE,
              "intermediate coarse grids must be multiples of 4 and at least 8 (16-colour smoother)");
      REQUIRE(b <= 64 && (64 % b) == 0, AMAMG_ERR_UNSUPPORTED_SHAPE,
              "intermediate coarse levels need a power-of-two block size <= 64");
    }
    REQUIRE(o * o * b <= 256, AMAMG_ERR_UNSUPPORTED_SHAPE, "coarse block size above 256");
    Lt /= a;
    Lx /= a;
    b *= o * o;
    if (k == 0) b += p.aug_vectors;     // the finest level's augmented coarse dofs
  }
  const LevelPlan& c = out.back();
  REQUIRE(int64_t(c.Lt) * c.Lx * c.b <= 4096, AMAMG_ERR_UNSUPPORTED_SHAPE,
          "coarsest level above 4096 unknowns (add a level)");
  REQUIRE(p.coarsest_tol == 0 || int64_t(c.Lt) * c.Lx * c.b <= kCoarsestGmresMaxN, AMAMG_ERR_UNSUPPORTED_SHAPE,
          "coarsest GMRES needs at most 2048 coarsest unknowns (add a level)");
  return out;
}

Geom make_geom(const LevelPlan& l, int a, int o, bool coarsest, int aug = 0) {
  Geom g{};
  g.Lt = l.Lt; g.Lx = l.Lx; g.b = l.b; g.a = a; g.o = o;
  g.nI = coarsest ? 0 : l.Lt / a;
  g.nJ = coarsest ? 0 : l.Lx / a;
  g.bv = o * o * l.b;
  g.bc = g.bv + (coarsest ? 0 : aug);
  return g;
}

Geom coarse_geom_of(const Geom& g) {
  Geom c{};
  c.Lt = g.nI; c.Lx = g.nJ; c.b = g.bc; c.a = g.a; c.o = g.o;
  return c;
}

}  // namespace

namespace amamg {
namespace rt {

size_t setup_bytes(int nt, int nx, const amamg_setup_params& p) {
  const auto plan = plan_levels(nt, nx, p);
  const int K = int(plan.size());
  const int a = p.agg_size, o = p.overlap;
  const int nv = (p.norm == AMAMG_NORM_TESTVEC) ? p.n_test_vectors : 0;
  const size_t c16 = sizeof(double2), c8 = sizeof(float2);
  size_t b = size_t(nt) * nx * 5 * 4 * c16;
  for (int k = 0; k + 1 < K; ++k) {
    const Geom g = make_geom(plan[k], a, o, false, k == 0 ? p.aug_vectors : 0);
    const Geom gc = make_geom(plan[k + 1], a, o, k + 1 == K - 1);
    const size_t nnode = g.nnode(), ndof = g.ndof(), ndc = gc.ndof(), nnc = gc.nnode();
    int nf = 0;
    const std::vector<int> tabs = footprint_tables(a, o, g.b, &nf);
    const size_t nW = size_t(g.nI) * g.nJ, nfd = size_t(nf) * g.b, ncol = g.ncol(), bc = g.bc;
    b += nnode * 9 + size_t(nv) * ndof * c16 + tabs.size() * 4 + nW * nf * g.b * 4 + nW * 4 * (1 + kDenseSolveInts);
    b += nW * nfd * (nfd + g.nvcol()) * c16 + ndof * ncol * (c16 + c8);
    if (k == 0 && p.aug_vectors > 0) b += size_t(nv) * ndof * c16 + nW * 4;
    if (k == 0) b += size_t(nv) * ndof * c16;                     // tv_alt
    b += size_t(nv) * ndc * c16 * 2;
    const size_t npc = size_t(probe_batch_colours(int(bc), period_of(gc.Lt) * period_of(gc.Lx))) * bc;
    b += npc * (2 * ndc + 2 * ndof) * c16 + npc * nW * restrict_chunks(g, nf, F64) * ncol * c16;
    if (k + 1 == K - 1) b += ndc * ndc * c16 * (p.coarsest_tol > 0 ? 5 : 4);
    else b += nnc * 25 * bc * bc * (c16 + c8) + nnc * bc * bc * (3 * c16 + c8) + nnc * 4 * kDenseSolveInts;
  }
  return b;
}

// ------------------------------------------------------------------------- GPU setup

// Buffers only the setup itself needs; with a scratch pool they live there (and are reused by
// the next setup) instead of in the hierarchy.
static bool setup_scratch(const char* name) {
  static const char* names[] = {"A0", "d_offs5", "d_offs25", "L_tv", "tv_alt", "Aug", "info", "Wc", "Ptv", "ainfo",
                                "pe", "py", "pz", "pu", "ppart", "Dg", "dinfo", "LUc", "cinfo", "keep"};
  for (const char* n : names)
    if (std::strcmp(n, name) == 0) return true;
  return false;
}

uint64_t next_generation() {
  static std::atomic<uint64_t> setups{0};   // unique over every hierarchy of the process
  return ++setups;
}

// Galerkin product of level k's operator (mass = false) or of its mass term (mass = true: the
// identity on level 0, G_k above) into `out` (level k + 1's stencil, or dense at the coarsest),
// by probing: for every colour class of coarse nodes (periods >= 5), P^H (Op (P e)) with unit
// vectors e on that class yields the blocks of the class's columns.
static void probe_galerkin(amamg_hierarchy* h, int k, bool mass, double2* out, hipStream_t s, Pool& tmp) {
  LevelData& L = h->lv[k];
  LevelData& C = h->lv[k + 1];
  const Geom& g = L.g;
  const Geom& gc = C.g;
  const bool dense = C.coarsest;
  const int bc = g.bc;
  const int64_t ndof = g.ndof(), ndof_c = gc.ndof();
  const int pt = period_of(gc.Lt), px = period_of(gc.Lx);
  amamg_gauge* gg = h->gauge;
  const double2* U0 = gg->U;
  const double2* U1 = gg->U + int64_t(gg->nt) * gg->nx;
  if (dense) HIPCHECK(hipMemsetAsync(out, 0, sizeof(double2) * ndof_c * ndof_c, s));
  else HIPCHECK(hipMemsetAsync(out, 0, sizeof(double2) * gc.nnode() * 25 * bc * bc, s));
  // the probe vectors of nb colours at once (at most 64 columns per batch): each column's
  // results are independent of the others in its batch
  const int ncolour = pt * px, nb = probe_batch_colours(bc, ncolour), nv = nb * bc;
  double2* pe = tmp.get<double2>("pe", k, size_t(nv) * ndof_c);
  double2* py = tmp.get<double2>("py", k, size_t(nv) * ndof);
  double2* pz = tmp.get<double2>("pz", k, size_t(nv) * ndof);
  double2* pu = tmp.get<double2>("pu", k, size_t(nv) * ndof_c);
  double2* ppart = tmp.get<double2>("ppart", k, size_t(nv) * g.nI * g.nJ * restrict_chunks(g, L.nf, F64) * g.ncol());
  for (int c0 = 0; c0 < ncolour; c0 += nb) {
    const int nc = std::min(nb, ncolour - c0), nvb = nc * bc;
    for (int q = 0; q < nc; ++q)
      probe_make(s, gc, pt, px, (c0 + q) / px, (c0 + q) % px, pe + size_t(q) * bc * ndof_c);
    prolong(s, F64, L.P, L.rows, L.nrows, L.nf, pe, py, g, 0, nvb, ndof, ndof_c, nullptr);
    const double2* r = pz;
    if (k == 0 && mass) r = py;
    else if (k == 0)
      wilson_apply(s, LINK_F64, U0, U1, F64, py, F64, pz, nullptr, g.Lt, g.Lx, h->m0, nvb, ndof, nullptr);
    else
      stencil_apply(s, F64, mass ? L.G : L.A, py, pz, nullptr, g.Lt, g.Lx, g.b, nvb, ndof, nullptr);
    restrict_(s, F64, L.P, L.rows, L.nrows, L.nf, F64, r, pu, ppart, g, nvb, ndof, ndof_c, nullptr);
    for (int q = 0; q < nc; ++q)
      probe_extract(s, gc, pt, px, (c0 + q) / px, (c0 + q) % px, pu + size_t(q) * bc * ndof_c, out, dense ? 1 : 0);
  }
  check_launch();
}

// Level k >= 1 from its operator: smoother blocks A_nn^-1 (non-coarsest) or the coarsest
// inverse (and its column-major copy for the GMRES variant).  Temporaries from `tmp`, the
// results from `keep` (where they are first allocated).
static void finish_level(amamg_hierarchy* h, int k, hipStream_t s, Pool& tmp, Pool& keep) {
  LevelData& C = h->lv[k];
  const Geom& gc = C.g;
  if (!C.coarsest) {
    const int bc = gc.b, nnc = gc.nnode();
    C.Dinv = keep.get<double2>("C_Dinv", k - 1, size_t(nnc) * bc * bc);
    double2* Dg = tmp.get<double2>("Dg", k - 1, size_t(nnc) * bc * 2 * bc);
    int* dinfo = tmp.get<int>("dinfo", k - 1, size_t(nnc) * kDenseSolveInts);
    aug_identity(s, C.A + 12 * bc * bc, int64_t(25) * bc * bc, bc, bc, Dg, nnc);
    dense_solve(s, Dg, bc, bc, nnc, dinfo);
    aug_extract(s, Dg, bc, bc, C.Dinv, nnc);
    check_launch();
    std::vector<int> hd(nnc);
    HIPCHECK(hipMemcpyAsync(hd.data(), dinfo, sizeof(int) * nnc, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    for (int n = 0; n < nnc; ++n)
      REQUIRE(hd[n] == 0, AMAMG_ERR_SINGULAR_LOCAL, "singular diagonal block on level " + std::to_string(k));
  } else {
    const int n = int(gc.ndof());
    double2* LUc = tmp.get<double2>("LUc", k - 1, size_t(n) * 2 * n);
    int* cinfo = tmp.get<int>("cinfo", k - 1, kDenseSolveInts);
    aug_identity(s, C.Adense, 0, n, n, LUc, 1);
    dense_solve(s, LUc, n, n, 1, cinfo);
    C.Ainv = h->mem.get<double2>("C_Ainv", k - 1, size_t(n) * n);
    aug_extract(s, LUc, n, n, C.Ainv, 1);
    check_launch();
    int hc = 0;
    HIPCHECK(hipMemcpyAsync(&hc, cinfo, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    REQUIRE(hc == 0, AMAMG_ERR_SINGULAR_COARSEST, "zero pivot in the coarsest factorisation");
    if (h->prm.coarsest_tol > 0) {
      C.Acm = h->mem.get<double2>("C_Acm", k - 1, size_t(n) * n);
      transpose_dense(s, C.Adense, C.Acm, n);
      check_launch();
    }
  }
}

// FP32 copies of level k's stencil and smoother blocks
static void cast_level(amamg_hierarchy* h, int k, hipStream_t s) {
  LevelData& L = h->lv[k];
  if (L.A) {
    const int64_t n = int64_t(L.g.nnode()) * 25 * L.g.b * L.g.b;
    L.A32 = h->mem.get<float2>("L_A32", k, n);
    cast_matrix(s, L.A, L.A32, n);
  }
  if (L.Dinv) {
    const int64_t n = int64_t(L.g.nnode()) * L.g.b * L.g.b;
    L.Dinv32 = h->mem.get<float2>("L_Dinv32", k, n);
    cast_matrix(s, L.Dinv, L.Dinv32, n);
  }
}

void run_setup(amamg_hierarchy* h, hipStream_t stream, Pool* scratch) {
  amamg_gauge* gg = h->gauge;
  hipStream_t s = stream ? stream : gg->ctx->stream;
  auto pool = [&](const char* name) -> Pool& { return scratch && setup_scratch(name) ? *scratch : h->mem; };
  const amamg_setup_params& p = h->prm;
  const auto plan = plan_levels(gg->nt, gg->nx, p);
  const int K = int(plan.size());
  const int a = p.agg_size, o = p.overlap;
  h->lv.resize(K);
  for (int k = 0; k < K; ++k) {
    h->lv[k].g = make_geom(plan[k], a, o, k == K - 1, k == 0 ? p.aug_vectors : 0);
    h->lv[k].coarsest = (k == K - 1);
  }
  const double2* U0 = gg->U;
  const double2* U1 = gg->U + int64_t(gg->nt) * gg->nx;
  const int nv = (p.norm == AMAMG_NORM_TESTVEC) ? p.n_test_vectors : 0;

  // fine operator in block-stencil form, used to gather the wirebasket systems
  double2* A0 = pool("A0").get<double2>("A0", -1, size_t(gg->nt) * gg->nx * 5 * 4);
  build_fine_stencil(s, U0, U1, gg->nt, gg->nx, h->m0, A0);
  const int offs5[10] = {0, 0, 1, 0, -1, 0, 0, 1, 0, -1};
  int offs25[50];
  for (int dt = -2, q = 0; dt <= 2; ++dt)
    for (int dx = -2; dx <= 2; ++dx, ++q) { offs25[2 * q] = dt; offs25[2 * q + 1] = dx; }
  int* d_offs5 = pool("d_offs5").get<int>("d_offs5", -1, 10);
  int* d_offs25 = pool("d_offs25").get<int>("d_offs25", -1, 50);
  HIPCHECK(hipMemcpyAsync(d_offs5, offs5, sizeof(offs5), hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(d_offs25, offs25, sizeof(offs25), hipMemcpyHostToDevice, s));

  double2* W = nullptr;   // test vectors entering level k
  for (int k = 0; k < K - 1; ++k) {
    LevelData& L = h->lv[k];
    const Geom& g = L.g;
    const int nnode = g.nnode();
    const int64_t ndof = g.ndof();
    L.kind = pool("L_kind").get<int8_t>("L_kind", k, nnode);
    L.owner = pool("L_owner").get<int>("L_owner", k, nnode);
    L.node = pool("L_node").get<int>("L_node", k, nnode);
    classify(s, g, L.kind, L.owner, L.node);
    check_launch();

    // test vectors: random at level 0, injected from the finer level otherwise; nu sweeps
    if (nv > 0) {
      L.tv = pool("L_tv").get<double2>("L_tv", k, size_t(nv) * ndof);
      if (k == 0) testvec_hash(s, p.seed, 0, nv, ndof, L.tv);
      else HIPCHECK(hipMemcpyAsync(L.tv, W, sizeof(double2) * nv * ndof, hipMemcpyDeviceToDevice, s));
      if (k == 0 && p.test_vector_sweeps > 0) {
        // two red-black sweeps per launch, between L_tv and a second buffer (bitwise the
        // colour-by-colour launches); the result ends in L_tv
        double2* alt = pool("tv_alt").get<double2>("tv_alt", k, size_t(nv) * ndof);
        double2* cur = L.tv;
        double2* nxt = alt;
        for (int sw = 0; sw < p.test_vector_sweeps; sw += 2) {
          const int ns = std::min(2, p.test_vector_sweeps - sw);
          wilson_gs_sweeps(s, LINK_F64, U0, U1, F64, cur, nxt, nullptr, g.Lt, g.Lx, h->m0, ns, nv, ndof, nullptr);
          std::swap(cur, nxt);
        }
        if (cur != L.tv)
          HIPCHECK(hipMemcpyAsync(L.tv, cur, sizeof(double2) * nv * ndof, hipMemcpyDeviceToDevice, s));
      } else {
        for (int sw = 0; sw < p.test_vector_sweeps; ++sw) {
          // the 16 colours as 4 colour blocks, one launch each for 8 x 8 blocks (one wave per node;
          // two colour-pair launches for other blocks); bitwise the colour-by-colour sweep
          for (int qb = 0; qb < 4; ++qb)
            stencil_gs_block(s, F64, L.A, L.Dinv, L.tv, nullptr, g.Lt, g.Lx, g.b, qb, nv, ndof, nullptr,
                             kGsNodeWaves, p.block_smoother);
        }
      }
      check_launch();
    }

    // local Schur-complement interpolation per wirebasket
    int nf = 0;
    const std::vector<int> tabs = footprint_tables(a, o, g.b, &nf);
    int* d_tabs = pool("d_tabs").get<int>("d_tabs", k, tabs.size());
    L.tabs = d_tabs;
    L.nf = nf;
    L.rows = pool("L_rows").get<int>("L_rows", k, size_t(g.nI) * g.nJ * nf * g.b);
    L.nrows = pool("L_nrows").get<int>("L_nrows", k, size_t(g.nI) * g.nJ);
    HIPCHECK(hipMemcpyAsync(d_tabs, tabs.data(), sizeof(int) * tabs.size(), hipMemcpyHostToDevice, s));
    owned_rows(s, g, d_tabs + g.fp(), nf, L.owner, L.rows, L.nrows);
    const int nW = g.nI * g.nJ, nfd = nf * g.b, ncol = g.ncol(), nvc = g.nvcol();
    double2* Aug = pool("Aug").get<double2>("Aug", k, size_t(nW) * nfd * (nfd + nvc));
    int* info = pool("info").get<int>("info", k, size_t(nW) * kDenseSolveInts);
    if (k == 0) gather_local(s, g, A0, 5, d_offs5, d_tabs, nf, Aug);
    else gather_local(s, g, L.A, 25, d_offs25, d_tabs, nf, Aug);
    dense_solve(s, Aug, nfd, nvc, nW, info);
    check_launch();
    std::vector<int> hinfo(nW);
    HIPCHECK(hipMemcpyAsync(hinfo.data(), info, sizeof(int) * nW, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    for (int w = 0; w < nW; ++w)
      REQUIRE(hinfo[w] == 0, AMAMG_ERR_SINGULAR_LOCAL,
              "zero pivot in the local system of wirebasket " + std::to_string(w) + " on level " + std::to_string(k));
    L.P = pool("L_P").get<double2>("L_P", k, size_t(ndof) * ncol);
    HIPCHECK(hipMemsetAsync(L.P, 0, sizeof(double2) * ndof * ncol, s));
    scatter_P(s, g, Aug, d_tabs, nf, L.owner, L.P);
    check_launch();

    // normalisation (and the test vectors handed to the next level)
    double2* Wc = nullptr;
    const Geom gc = coarse_geom_of(g);
    const int64_t ndof_c = gc.ndof();
    if (nv > 0) {
      Wc = pool("Wc").get<double2>("Wc", k, size_t(nv) * ndof_c);
      HIPCHECK(hipMemsetAsync(Wc, 0, sizeof(double2) * nv * ndof_c, s));
      inject(s, g, L.node, L.kind, L.tv, Wc, nv);
    }
    normalise(s, g, L.P, L.owner, L.tv, Wc, nv, p.norm);
    check_launch();
    if (k == 0 && p.aug_vectors > 0) {
      // augmented coarse space: the test vectors' residuals of the wirebasket interpolation
      REQUIRE(nf * g.b <= kAugMaxRows, AMAMG_ERR_UNSUPPORTED_SHAPE,
              "augmented coarse space: wirebaskets own at most 1024 rows");
      double2* Ptv = pool("Ptv").get<double2>("Ptv", k, size_t(nv) * ndof);
      int* ainfo = pool("ainfo").get<int>("ainfo", k, nW);
      prolong(s, F64, L.P, L.rows, L.nrows, L.nf, Wc, Ptv, g, 0, nv, ndof, ndof_c, nullptr);
      augment(s, g, L.P, L.rows, L.nrows, nf * g.b, L.tv, Ptv, Wc, nv, p.aug_vectors, ainfo);
      check_launch();
      std::vector<int> ha(nW);
      HIPCHECK(hipMemcpyAsync(ha.data(), ainfo, sizeof(int) * nW, hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      for (int w = 0; w < nW; ++w)
        REQUIRE(ha[w] == 0, AMAMG_ERR_SINGULAR_LOCAL,
                "a test vector's interpolation residual vanishes on wirebasket " + std::to_string(w));
    }

    // Galerkin operator by probing
    LevelData& C = h->lv[k + 1];
    const bool dense = C.coarsest;
    const int bc = g.bc;
    const int nnc = gc.nnode();
    if (dense) C.Adense = h->mem.get<double2>("C_Adense", k, size_t(ndof_c) * ndof_c);
    else C.A = pool("C_A").get<double2>("C_A", k, size_t(nnc) * 25 * bc * bc);
    probe_galerkin(h, k, false, dense ? C.Adense : C.A, s, pool("pe"));
    finish_level(h, k + 1, s, pool("Dg"), pool("C_Dinv"));
    W = Wc;
    // the next level's test vectors must outlive this iteration's temporaries
    if (nv > 0 && !dense) {
      double2* keep = pool("keep").get<double2>("keep", k, size_t(nv) * ndof_c);
      HIPCHECK(hipMemcpyAsync(keep, Wc, sizeof(double2) * nv * ndof_c, hipMemcpyDeviceToDevice, s));
      W = keep;
    }
  }

  // FP32 copies for the mixed-precision V-cycle
  for (int k = 0; k < K; ++k) {
    LevelData& L = h->lv[k];
    if (L.P) {
      const int64_t n = L.g.ndof() * L.g.ncol();
      L.P32 = pool("L_P32").get<float2>("L_P32", k, n);
      cast_matrix(s, L.P, L.P32, n);
    }
    cast_level(h, k, s);
  }
  check_launch();
  HIPCHECK(hipStreamSynchronize(s));
  h->generation = next_generation();
  h->mass_terms = false;
  if (scratch)
    for (LevelData& L : h->lv) L.tv = nullptr;
}

void ensure_mass_terms(amamg_hierarchy* h, hipStream_t stream) {
  if (h->mass_terms) return;
  hipStream_t s = stream ? stream : h->gauge->ctx->stream;
  const int K = int(h->lv.size());
  Pool tmp;   // probing temporaries, freed on return
  // G_{k+1} = P_k^H G_k P_k with G_0 = I: the Galerkin images of the mass term
  for (int k = 0; k + 1 < K; ++k) {
    LevelData& C = h->lv[k + 1];
    const Geom& gc = C.g;
    const size_t cnt = C.coarsest ? size_t(gc.ndof()) * gc.ndof() : size_t(gc.nnode()) * 25 * gc.b * gc.b;
    C.G = h->mem.get<double2>("C_G", k, cnt);
    probe_galerkin(h, k, true, C.G, s, tmp);
  }
  HIPCHECK(hipStreamSynchronize(s));
  h->mass_terms = true;
}

size_t derive_bytes(const amamg_hierarchy* h) {
  size_t b = 0;
  for (size_t k = 1; k < h->lv.size(); ++k) {
    const Geom& gc = h->lv[k].g;
    if (h->lv[k].coarsest) {
      const size_t n = size_t(gc.ndof());
      // matrix, inverse, column-major copy (GMRES variant), LU workspace [n][2n]
      b += n * n * 16 * (h->prm.coarsest_tol > 0 ? 5 : 4);
    } else {
      const size_t nb = size_t(gc.nnode()) * gc.b * gc.b;
      b += nb * 25 * (16 + 8) + nb * (16 + 8) + nb * 2 * 16 + size_t(gc.nnode()) * 4;
    }
  }
  return b;
}

amamg_hierarchy* derive_mass(amamg_hierarchy* base, double m0, hipStream_t stream) {
  REQUIRE(base->mass_terms, AMAMG_ERR_INVALID_ARG, "internal: derive_mass needs the base's mass terms");
  hipStream_t s = stream ? stream : base->gauge->ctx->stream;
  std::unique_ptr<amamg_hierarchy> h(new amamg_hierarchy());
  h->gauge = base->gauge;
  h->prm = base->prm;
  h->m0 = base->m0;
  h->lv = base->lv;            // wirebaskets, interpolation, mass terms: shared
  h->mass_terms = true;
  // own copies of the operators at the base's mass; everything derived from them is rebuilt
  for (size_t k = 1; k < h->lv.size(); ++k) {
    LevelData& C = h->lv[k];
    const Geom& gc = C.g;
    if (C.coarsest) {
      const size_t cnt = size_t(gc.ndof()) * gc.ndof();
      C.Adense = h->mem.get<double2>("C_Adense", int(k) - 1, cnt);
      HIPCHECK(hipMemcpyAsync(C.Adense, base->lv[k].Adense, sizeof(double2) * cnt, hipMemcpyDeviceToDevice, s));
      C.Ainv = C.Acm = nullptr;
    } else {
      const size_t cnt = size_t(gc.nnode()) * 25 * gc.b * gc.b;
      C.A = h->mem.get<double2>("C_A", int(k) - 1, cnt);
      HIPCHECK(hipMemcpyAsync(C.A, base->lv[k].A, sizeof(double2) * cnt, hipMemcpyDeviceToDevice, s));
      C.A32 = nullptr;
      C.Dinv = nullptr;
      C.Dinv32 = nullptr;
    }
  }
  shift_mass(h.get(), m0, s);
  h->base = base;                 // the caller counts it in base->derived and gauge->nhier
  return h.release();
}

void shift_mass(amamg_hierarchy* h, double m0, hipStream_t stream) {
  hipStream_t s = stream ? stream : h->gauge->ctx->stream;
  const int K = int(h->lv.size());
  Pool tmp;   // factorisation temporaries, freed on return
  ensure_mass_terms(h, s);
  const double dm = m0 - h->m0;
  h->m0 = m0;
  // the fine operator takes m0 directly; every coarser one moves by dm times its mass term
  for (int k = 1; k < K; ++k) {
    LevelData& C = h->lv[k];
    const Geom& gc = C.g;
    if (C.coarsest) axpy_real(s, C.Adense, dm, C.G, int64_t(gc.ndof()) * gc.ndof());
    else axpy_real(s, C.A, dm, C.G, int64_t(gc.nnode()) * 25 * gc.b * gc.b);
  }
  check_launch();
  h->generation = next_generation();     // before the checks: a failed move still invalidates graphs
  for (int k = 1; k < K; ++k) {
    finish_level(h, k, s, tmp, h->mem);
    cast_level(h, k, s);
  }
  check_launch();
  HIPCHECK(hipStreamSynchronize(s));
}

}  // namespace rt
}  // namespace amamg

// ---------------------------------------------------------------------------------- ABI

extern "C" {

void amamg_default_setup_params(amamg_setup_params* p) {
  if (!p) return;
  p->levels = 2; p->agg_size = 4; p->overlap = 1; p->n_test_vectors = 4;
  p->test_vector_sweeps = 4; p->pre_sweeps = 0; p->post_sweeps = 2;
  p->norm = AMAMG_NORM_TESTVEC; p->seed = 0;
  p->coarsest_tol = 0; p->coarsest_max_iters = 32; p->block_smoother = 0;
  p->aug_vectors = 0; p->reserved = 0;
}

void amamg_default_solve_params(amamg_solve_params* p) {
  if (!p) return;
  p->restart = 20; p->max_iters = 10000; p->rel_tol = 1e-10; p->precision = AMAMG_FP64;
  p->use_initial_guess = 0;
  p->groups = 1;
  p->graphs = 0;
}

amamg_status amamg_context_create(int device, void* hip_stream, amamg_context** out) {
  if (!out) return AMAMG_ERR_INVALID_ARG;
  *out = nullptr;
  amamg_context* c = new amamg_context();
  try {
    int ndev = 0;
    HIPCHECK(hipGetDeviceCount(&ndev));
    REQUIRE(device >= 0 && device < ndev, AMAMG_ERR_INVALID_ARG, "no such device");
    HIPCHECK(hipSetDevice(device));
    c->device = device;
    noalloc_init(device);
    if (hip_stream) {
      c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      HIPCHECK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
  } catch (const Fail& f) {
    delete c;
    return f.code;
  }
  *out = c;
  return AMAMG_OK;
}

amamg_status amamg_context_destroy(amamg_context* ctx) {
  if (!ctx) return AMAMG_ERR_INVALID_ARG;
  for (hipEvent_t e : ctx->timer.events) (void)hipEventDestroy(e);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return AMAMG_OK;
}

const char* amamg_last_error(const amamg_context* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

amamg_status amamg_gauge_load(amamg_context* ctx, int32_t nt, int32_t nx, const double* links,
                              double m0, amamg_gauge** out) {
  if (!ctx || !out || !links) return ctx ? fail(ctx, {AMAMG_ERR_INVALID_ARG, "null argument"}) : AMAMG_ERR_INVALID_ARG;
  *out = nullptr;
  amamg_gauge* g = new amamg_gauge();
  try {
    REQUIRE(nt >= 4 && nx >= 4 && nt % 2 == 0 && nx % 2 == 0, AMAMG_ERR_UNSUPPORTED_SHAPE,
            "lattice sizes must be even and >= 4");
    REQUIRE(int64_t(nt) * nx <= (int64_t(1) << 28), AMAMG_ERR_UNSUPPORTED_SHAPE, "lattice too large");
    const size_t nval = size_t(2) * nt * nx * 2;
    REQUIRE(std::isfinite(m0) && finite_all(links, nval), AMAMG_ERR_NONFINITE, "non-finite link or mass");
    HIPCHECK(hipSetDevice(ctx->device));
    g->ctx = ctx; g->nt = nt; g->nx = nx; g->m0 = m0;
    g->U = g->mem.alloc<double2>(size_t(2) * nt * nx);
    HIPCHECK(hipMemcpyAsync(g->U, links, sizeof(double) * nval, hipMemcpyHostToDevice, ctx->stream));
    HIPCHECK(hipStreamSynchronize(ctx->stream));
  } catch (const Fail& f) {
    delete g;
    return fail(ctx, f);
  }
  *out = g;
  return AMAMG_OK;
}

amamg_status amamg_gauge_set_mass(amamg_gauge* g, double m0) {
  if (!g) return AMAMG_ERR_INVALID_ARG;
  if (!std::isfinite(m0)) return fail(g->ctx, {AMAMG_ERR_NONFINITE, "non-finite mass"});
  g->m0 = m0;
  return AMAMG_OK;
}

amamg_status amamg_gauge_update_links(amamg_gauge* g, const double* links) {
  if (!g || !links) return g ? fail(g->ctx, {AMAMG_ERR_INVALID_ARG, "null argument"}) : AMAMG_ERR_INVALID_ARG;
  amamg_context* ctx = g->ctx;
  try {
    const size_t nval = size_t(2) * g->nt * g->nx * 2;
    REQUIRE(finite_all(links, nval), AMAMG_ERR_NONFINITE, "non-finite link");
    HIPCHECK(hipSetDevice(ctx->device));
    HIPCHECK(hipMemcpyAsync(g->U, links, sizeof(double) * nval, hipMemcpyHostToDevice, ctx->stream));
    HIPCHECK(hipStreamSynchronize(ctx->stream));
    g->version += 1;
  } catch (const Fail& f) {
    return fail(ctx, f);
  }
  return AMAMG_OK;
}

amamg_status amamg_gauge_destroy(amamg_gauge* g) {
  if (!g) return AMAMG_ERR_INVALID_ARG;
  if (g->nhier > 0) return fail(g->ctx, {AMAMG_ERR_INVALID_ARG, "gauge still used by hierarchies"});
  delete g;
  return AMAMG_OK;
}

amamg_status amamg_setup(amamg_gauge* g, const amamg_setup_params* params, amamg_hierarchy** out) {
  if (!g || !out) return g ? fail(g->ctx, {AMAMG_ERR_INVALID_ARG, "null argument"}) : AMAMG_ERR_INVALID_ARG;
  *out = nullptr;
  amamg_hierarchy* h = new amamg_hierarchy();
  h->gauge = g;
  h->m0 = g->m0;
  if (params) h->prm = *params;
  else amamg_default_setup_params(&h->prm);
  try {
    HIPCHECK(hipSetDevice(g->ctx->device));
    run_setup(h);
  } catch (const Fail& f) {
    delete h;
    return fail(g->ctx, f);
  }
  g->nhier += 1;
  *out = h;
  return AMAMG_OK;
}

amamg_status amamg_hierarchy_update(amamg_hierarchy* h) {
  if (!h) return AMAMG_ERR_INVALID_ARG;
  amamg_gauge* g = h->gauge;
  if (h->derived > 0) return fail(g->ctx, {AMAMG_ERR_INVALID_ARG, "hierarchies derived from this one still exist"});
  if (h->base) return fail(g->ctx, {AMAMG_ERR_INVALID_ARG, "a derived hierarchy follows its base: derive it again"});
  try {
    HIPCHECK(hipSetDevice(g->ctx->device));
    h->m0 = g->m0;
    run_setup(h);
  } catch (const Fail& f) {
    return fail(g->ctx, f);
  }
  return AMAMG_OK;
}

amamg_status amamg_hierarchy_set_mass(amamg_hierarchy* h, double m0) {
  if (!h) return AMAMG_ERR_INVALID_ARG;
  amamg_gauge* g = h->gauge;
  if (!std::isfinite(m0)) return fail(g->ctx, {AMAMG_ERR_INVALID_ARG, "mass must be finite"});
  if (h->derived > 0) return fail(g->ctx, {AMAMG_ERR_INVALID_ARG, "hierarchies derived from this one still exist"});
  try {
    HIPCHECK(hipSetDevice(g->ctx->device));
    shift_mass(h, m0);
  } catch (const Fail& f) {
    return fail(g->ctx, f);
  }
  return AMAMG_OK;
}

amamg_status amamg_hierarchy_derive_mass(amamg_hierarchy* base, double m0, amamg_hierarchy** out) {
  if (!base || !out) return base ? fail(base->gauge->ctx, {AMAMG_ERR_INVALID_ARG, "null argument"}) : AMAMG_ERR_INVALID_ARG;
  *out = nullptr;
  amamg_gauge* g = base->gauge;
  if (!std::isfinite(m0)) return fail(g->ctx, {AMAMG_ERR_INVALID_ARG, "mass must be finite"});
  if (base->base) return fail(g->ctx, {AMAMG_ERR_INVALID_ARG, "derive from the base hierarchy, not a derived one"});
  try {
    HIPCHECK(hipSetDevice(g->ctx->device));
    ensure_mass_terms(base);
    *out = derive_mass(base, m0);
    base->derived += 1;
    g->nhier += 1;
  } catch (const Fail& f) {
    return fail(g->ctx, f);
  }
  return AMAMG_OK;
}

amamg_status amamg_hierarchy_destroy(amamg_hierarchy* h) {
  if (!h) return AMAMG_ERR_INVALID_ARG;
  if (h->derived > 0) return fail(h->gauge->ctx, {AMAMG_ERR_INVALID_ARG, "hierarchies derived from this one still exist"});
  if (h->base) h->base->derived -= 1;
  h->gauge->nhier -= 1;
  delete h;
  return AMAMG_OK;
}

amamg_status amamg_solve_multi_device(amamg_hierarchy* const* hs, int32_t nlat, const int32_t* nrhs,
                                      const void* const* psi_dev, void* const* x_dev,
                                      const amamg_solve_params* params, amamg_solve_info* info,
                                      void* hip_stream) {
  if (!hs || nlat < 1 || !hs[0]) return AMAMG_ERR_INVALID_ARG;
  amamg_context* ctx = hs[0]->gauge->ctx;
  if (!nrhs || !psi_dev || !x_dev) return fail(ctx, {AMAMG_ERR_INVALID_ARG, "null argument"});
  std::vector<amamg_hierarchy*> h(nlat);
  std::vector<int> nr(nlat);
  std::vector<const double2*> b(nlat);
  std::vector<double2*> x(nlat);
  for (int l = 0; l < nlat; ++l) {
    if (!hs[l] || !psi_dev[l] || !x_dev[l]) return fail(ctx, {AMAMG_ERR_INVALID_ARG, "null hierarchy or field pointer"});
    if (!aligned16(psi_dev[l]) || !aligned16(x_dev[l]))
      return fail(ctx, {AMAMG_ERR_INVALID_ARG, "field pointers must be 16-byte aligned"});
    h[l] = hs[l];
    nr[l] = nrhs[l];
    b[l] = static_cast<const double2*>(psi_dev[l]);
    x[l] = static_cast<double2*>(x_dev[l]);
  }
  amamg_solve_params p;
  if (params) p = *params;
  else amamg_default_solve_params(&p);
  try {
    HIPCHECK(hipSetDevice(ctx->device));
    const hipStream_t root = hip_stream ? static_cast<hipStream_t>(hip_stream) : ctx->stream;
    const amamg_status st = run_solve_multi(h, nr, b, x, p, info, root);
    if (st == AMAMG_NOT_CONVERGED) ctx->err = "not converged within max_iters";
    return st;
  } catch (const Fail& f) {
    return fail(ctx, f);
  }
}

amamg_status amamg_solve_device(amamg_hierarchy* h, int32_t nrhs, const void* psi_dev, void* x_dev,
                                const amamg_solve_params* params, amamg_solve_info* info, void* hip_stream) {
  if (!h) return AMAMG_ERR_INVALID_ARG;
  amamg_context* ctx = h->gauge->ctx;
  if (!psi_dev || !x_dev) return fail(ctx, {AMAMG_ERR_INVALID_ARG, "null field pointer"});
  if (!aligned16(psi_dev) || !aligned16(x_dev))
    return fail(ctx, {AMAMG_ERR_INVALID_ARG, "field pointers must be 16-byte aligned"});
  amamg_solve_params p;
  if (params) p = *params;
  else amamg_default_solve_params(&p);
  hipEvent_t ready = nullptr;
  try {
    HIPCHECK(hipSetDevice(ctx->device));
    const hipStream_t caller = static_cast<hipStream_t>(hip_stream);
    if (caller && caller != ctx->stream) {
      // the solve reads psi and x0 after the work the caller queued on its stream
      HIPCHECK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
      HIPCHECK(hipEventRecord(ready, caller));
      HIPCHECK(hipStreamWaitEvent(ctx->stream, ready, 0));
    }
    const amamg_status st = run_solve(h, nrhs, static_cast<const double2*>(psi_dev), static_cast<double2*>(x_dev), p, info);
    if (ready) (void)hipEventDestroy(ready);
    return st;
  } catch (const Fail& f) {
    if (ready) (void)hipEventDestroy(ready);
    return fail(ctx, f);
  }
}

amamg_status amamg_solve(amamg_hierarchy* h, int32_t nrhs, const double* psi, double* x,
                         const amamg_solve_params* params, amamg_solve_info* info) {
  if (!h) return AMAMG_ERR_INVALID_ARG;
  amamg_context* ctx = h->gauge->ctx;
  if (!psi || !x || nrhs < 1) return fail(ctx, {AMAMG_ERR_INVALID_ARG, "null field pointer or nrhs < 1"});
  amamg_solve_params p;
  if (params) p = *params;
  else amamg_default_solve_params(&p);
  const size_t bytes = sizeof(double2) * size_t(nrhs) * h->lv[0].g.ndof();
  Arena io;
  try {
    HIPCHECK(hipSetDevice(ctx->device));
    double2* db = io.alloc<double2>(bytes / sizeof(double2));
    double2* dx = io.alloc<double2>(bytes / sizeof(double2));
    HIPCHECK(hipMemcpyAsync(db, psi, bytes, hipMemcpyHostToDevice, ctx->stream));
    if (p.use_initial_guess) HIPCHECK(hipMemcpyAsync(dx, x, bytes, hipMemcpyHostToDevice, ctx->stream));
    amamg_status st = run_solve(h, nrhs, db, dx, p, info);
    HIPCHECK(hipMemcpyAsync(x, dx, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(hipStreamSynchronize(ctx->stream));
    return st;
  } catch (const Fail& f) {
    return fail(ctx, f);
  }
}

amamg_status amamg_residual_history(const amamg_hierarchy* h, int32_t rhs, double* out, int32_t capacity,
                                    int32_t* n_written, int32_t* is_true) {
  if (!h || rhs < 0 || rhs >= int(h->history.size())) return AMAMG_ERR_INVALID_ARG;
  const auto& v = h->history[rhs];
  if (n_written) *n_written = int32_t(v.size());
  const int nw = std::min<int>(capacity, int(v.size()));
  for (int i = 0; i < nw; ++i) {
    if (out) out[i] = v[i].x;
    if (is_true) is_true[i] = v[i].y != 0.0;
  }
  return AMAMG_OK;
}

amamg_status amamg_context_set_tuning(amamg_context* ctx, int32_t mode, int32_t force) {
  if (!ctx) return AMAMG_ERR_INVALID_ARG;
  if (mode < AMAMG_TUNE_AUTO || mode > AMAMG_TUNE_FORCE) return fail(ctx, {AMAMG_ERR_INVALID_ARG, "unknown tuning mode"});
  std::lock_guard<std::mutex> lk(ctx->tuner.mu);
  ctx->tuner.mode = mode;
  ctx->tuner.force = force;
  return AMAMG_OK;
}

amamg_status amamg_tuning_entries(amamg_context* ctx, amamg_tune_entry* out, int32_t cap, int32_t* count) {
  if (!ctx || !count || cap < 0 || (cap > 0 && !out)) return AMAMG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(ctx->tuner.mu);
  int32_t i = 0;
  for (const auto& kv : ctx->tuner.entries) {
    if (i < cap) {
      amamg_tune_entry& e = out[i];
      e = amamg_tune_entry{};
      e.kind = kv.first[0]; e.lt = kv.first[1]; e.lx = kv.first[2]; e.b = kv.first[3];
      e.precision = kv.first[4]; e.nrhs = kv.first[5];
      e.choice = kv.second.choice;
      e.ncand = int32_t(std::min<size_t>(8, kv.second.cand.size()));
      for (int q = 0; q < e.ncand; ++q) {
        e.cand[q] = kv.second.cand[q];
        e.us[q] = q < int(kv.second.us.size()) ? kv.second.us[q] : 0.0;
      }
    }
    ++i;
  }
  *count = i;
  return AMAMG_OK;
}

amamg_status amamg_apply_dirac(amamg_gauge* g, int32_t precision, int32_t nrhs, const double* in,
                               double* out) {
  if (!g || !in || !out || nrhs < 1) return g ? fail(g->ctx, {AMAMG_ERR_INVALID_ARG, "bad argument"}) : AMAMG_ERR_INVALID_ARG;
  amamg_context* ctx = g->ctx;
  try {
    REQUIRE(precision == AMAMG_FP64 || precision == AMAMG_MIXED_FP32, AMAMG_ERR_INVALID_ARG,
            "precision must be FP64 or MIXED_FP32");
    HIPCHECK(hipSetDevice(ctx->device));
    const int64_t n = int64_t(g->nt) * g->nx * 2;
    Arena io;
    double2* dx = io.alloc<double2>(size_t(nrhs) * n);
    double2* dy = io.alloc<double2>(size_t(nrhs) * n);
    HIPCHECK(hipMemcpyAsync(dx, in, sizeof(double2) * nrhs * n, hipMemcpyHostToDevice, ctx->stream));
    LinkStore ls = precision == AMAMG_FP64 ? LINK_F64 : LINK_F32;
    ensure_links(g, ls);
    wilson_apply(ctx->stream, ls, link0(g, ls), link1(g, ls), F64, dx, F64, dy, nullptr, g->nt, g->nx,
                 g->m0, nrhs, n, nullptr);
    check_launch();
    HIPCHECK(hipMemcpyAsync(out, dy, sizeof(double2) * nrhs * n, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(hipStreamSynchronize(ctx->stream));
  } catch (const Fail& f) {
    return fail(ctx, f);
  }
  return AMAMG_OK;
}

amamg_status amamg_dense_solve(amamg_context* ctx, int32_t n, int32_t nrhs, int32_t nsys, double* aug,
                               int32_t* info) {
  if (!ctx) return AMAMG_ERR_INVALID_ARG;
  if (!aug || !info || n < 1 || nrhs < 1 || nsys < 1)
    return fail(ctx, {AMAMG_ERR_INVALID_ARG, "dense solve: null pointer or a size below 1"});
  try {
    HIPCHECK(hipSetDevice(ctx->device));
    const size_t count = size_t(nsys) * n * (size_t(n) + nrhs);
    Arena io;
    double2* d = io.alloc<double2>(count);
    int* di = io.alloc<int>(size_t(nsys) * kDenseSolveInts);
    HIPCHECK(hipMemcpyAsync(d, aug, sizeof(double2) * count, hipMemcpyHostToDevice, ctx->stream));
    dense_solve(ctx->stream, d, n, nrhs, nsys, di);
    check_launch();
    HIPCHECK(hipMemcpyAsync(aug, d, sizeof(double2) * count, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(hipMemcpyAsync(info, di, sizeof(int) * nsys, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(hipStreamSynchronize(ctx->stream));
  } catch (const Fail& f) {
    return fail(ctx, f);
  }
  return AMAMG_OK;
}

amamg_status amamg_apply_dirac_device(amamg_gauge* g, int32_t precision, int32_t nrhs,
                                      const void* in_dev, void* out_dev) {
  if (!g || !in_dev || !out_dev || nrhs < 1)
    return g ? fail(g->ctx, {AMAMG_ERR_INVALID_ARG, "bad argument"}) : AMAMG_ERR_INVALID_ARG;
  amamg_context* ctx = g->ctx;
  try {
    REQUIRE(precision >= AMAMG_FP64 && precision <= AMAMG_MIXED_FP32_BF16LINKS, AMAMG_ERR_INVALID_ARG,
            "unknown precision");
    REQUIRE(aligned16(in_dev) && aligned16(out_dev), AMAMG_ERR_INVALID_ARG,
            "field pointers must be 16-byte aligned");
    HIPCHECK(hipSetDevice(ctx->device));
    const int64_t n = int64_t(g->nt) * g->nx * 2;
    const LinkStore ls = precision == AMAMG_FP64 ? LINK_F64 : precision == AMAMG_MIXED_FP32 ? LINK_F32 : LINK_BF16;
    const Real v = precision == AMAMG_FP64 ? F64 : F32;
    ensure_links(g, ls);
    wilson_apply(ctx->stream, ls, link0(g, ls), link1(g, ls), v, in_dev, v, out_dev, nullptr, g->nt,
                 g->nx, g->m0, nrhs, n, nullptr);
    check_launch();
  } catch (const Fail& f) {
    return fail(ctx, f);
  }
  return AMAMG_OK;
}

amamg_status amamg_kernel_timer(amamg_context* ctx, uint32_t family_mask) {
  if (!ctx || (family_mask & 1u) || family_mask >= (1u << KernelTimer::NF)) return AMAMG_ERR_INVALID_ARG;
  KernelTimer& t = ctx->timer;
  t.mask = family_mask;
  t.pending.clear();
  for (int f = 0; f < KernelTimer::NF; ++f) {
    t.launches[f] = 0;
    t.total_ms[f] = 0.0;
    t.total_bytes[f] = 0.0;
  }
  return AMAMG_OK;
}

amamg_status amamg_kernel_timer_read(const amamg_context* ctx, int32_t family, int64_t* launches,
                                     double* total_ms, double* algorithmic_bytes) {
  if (!ctx || family <= 0 || family >= KernelTimer::NF) return AMAMG_ERR_INVALID_ARG;
  if (launches) *launches = ctx->timer.launches[family];
  if (total_ms) *total_ms = ctx->timer.total_ms[family];
  if (algorithmic_bytes) *algorithmic_bytes = ctx->timer.total_bytes[family];
  return AMAMG_OK;
}

amamg_status amamg_level_info(const amamg_hierarchy* h, int32_t level, int32_t* lt, int32_t* lx,
                              int32_t* b) {
  if (!h || level < 0 || level >= int(h->lv.size())) return AMAMG_ERR_INVALID_ARG;
  const Geom& g = h->lv[level].g;
  if (lt) *lt = g.Lt;
  if (lx) *lx = g.Lx;
  if (b) *b = g.b;
  return AMAMG_OK;
}

static amamg_status copy_out(const amamg_hierarchy* h, void* dst, const void* src, size_t bytes) {
  amamg_context* ctx = h->gauge->ctx;
  try {
    HIPCHECK(hipSetDevice(ctx->device));
    HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(hipStreamSynchronize(ctx->stream));
  } catch (const Fail& f) {
    return fail(ctx, f);
  }
  return AMAMG_OK;
}

amamg_status amamg_get_aggregates(const amamg_hierarchy* h, int32_t level, int8_t* kind,
                                  int32_t* owner, int32_t* node) {
  if (!h || level < 0 || level >= int(h->lv.size()) - 1) return AMAMG_ERR_INVALID_ARG;
  const LevelData& L = h->lv[level];
  const size_t nn = L.g.nnode();
  amamg_status s = AMAMG_OK;
  if (kind && (s = copy_out(h, kind, L.kind, nn)) != AMAMG_OK) return s;
  if (owner && (s = copy_out(h, owner, L.owner, nn * 4)) != AMAMG_OK) return s;
  if (node && (s = copy_out(h, node, L.node, nn * 4)) != AMAMG_OK) return s;
  return AMAMG_OK;
}

amamg_status amamg_get_prolongator(const amamg_hierarchy* h, int32_t level, double* out) {
  if (!h || !out || level < 0 || level >= int(h->lv.size()) - 1) return AMAMG_ERR_INVALID_ARG;
  const LevelData& L = h->lv[level];
  return copy_out(h, out, L.P, sizeof(double2) * L.g.ndof() * L.g.ncol());
}

amamg_status amamg_get_coarse_operator(const amamg_hierarchy* h, int32_t level, double* out) {
  if (!h || !out || level < 1 || level >= int(h->lv.size())) return AMAMG_ERR_INVALID_ARG;
  const LevelData& L = h->lv[level];
  if (L.coarsest) return copy_out(h, out, L.Adense, sizeof(double2) * L.g.ndof() * L.g.ndof());
  return copy_out(h, out, L.A, sizeof(double2) * L.g.nnode() * 25 * L.g.b * L.g.b);
}

amamg_status amamg_apply_transfer(amamg_hierarchy* h, int32_t level, int32_t precision, int32_t direction,
                                  int32_t nrhs, const double* in, double* out) {
  if (!h || !in || !out || nrhs < 1) return h ? fail(h->gauge->ctx, {AMAMG_ERR_INVALID_ARG, "bad argument"}) : AMAMG_ERR_INVALID_ARG;
  amamg_context* ctx = h->gauge->ctx;
  try {
    REQUIRE(precision == AMAMG_FP64 || precision == AMAMG_MIXED_FP32, AMAMG_ERR_INVALID_ARG,
            "precision must be FP64 or MIXED_FP32");
    REQUIRE(level >= 0 && level + 1 < int(h->lv.size()), AMAMG_ERR_INVALID_ARG,
            "level must have a coarser level");
    REQUIRE(direction == 0 || direction == 1, AMAMG_ERR_INVALID_ARG, "direction must be 0 or 1");
    HIPCHECK(hipSetDevice(ctx->device));
    const LevelData& L = h->lv[level];
    const Geom& g = L.g;
    const int64_t nd = g.ndof(), ndc = h->lv[level + 1].g.ndof();
    const bool f64 = precision == AMAMG_FP64;
    const Real T = f64 ? F64 : F32;
    const void* P = f64 ? (const void*)L.P : (const void*)L.P32;
    const size_t cs = f64 ? sizeof(double2) : sizeof(float2);
    const int64_t nin = direction == 0 ? nd : ndc, nout = direction == 0 ? ndc : nd;
    hipStream_t s = ctx->stream;
    Arena io;
    // inputs: FP64 for the restriction (the fine level's restriction reads the FP64 Krylov
    // vector), the level's precision for the prolongation; outputs in the level's precision
    std::vector<float2> h32;
    void* din = nullptr;
    if (direction == 0 || f64) {
      din = io.alloc<double2>(size_t(nrhs) * nin);
      HIPCHECK(hipMemcpyAsync(din, in, sizeof(double2) * nrhs * nin, hipMemcpyHostToDevice, s));
    } else {
      h32.resize(size_t(nrhs) * nin);
      for (size_t i = 0; i < h32.size(); ++i) h32[i] = make_float2(float(in[2 * i]), float(in[2 * i + 1]));
      din = io.alloc<float2>(h32.size());
      HIPCHECK(hipMemcpyAsync(din, h32.data(), sizeof(float2) * h32.size(), hipMemcpyHostToDevice, s));
    }
    void* dout = io.alloc<char>(cs * nrhs * nout);
    if (direction == 0) {
      void* part = io.alloc<char>(cs * nrhs * g.nI * g.nJ * restrict_chunks(g, L.nf, T) * g.ncol());
      restrict_(s, T, P, L.rows, L.nrows, L.nf, F64, din, dout, part, g, nrhs, nd, ndc, nullptr);
    } else {
      prolong(s, T, P, L.rows, L.nrows, L.nf, din, dout, g, 0, nrhs, nd, ndc, nullptr);
    }
    check_launch();
    if (f64) {
      HIPCHECK(hipMemcpyAsync(out, dout, sizeof(double2) * nrhs * nout, hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
    } else {
      std::vector<float2> o32(size_t(nrhs) * nout);
      HIPCHECK(hipMemcpyAsync(o32.data(), dout, sizeof(float2) * o32.size(), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      for (size_t i = 0; i < o32.size(); ++i) { out[2 * i] = o32[i].x; out[2 * i + 1] = o32[i].y; }
    }
  } catch (const Fail& f) {
    return fail(ctx, f);
  }
  return AMAMG_OK;
}

amamg_status amamg_apply_smoother(amamg_hierarchy* h, int32_t level, int32_t precision, int32_t nrhs,
                                  int32_t sweeps, const double* f, double* x) {
  if (!h || !f || !x || nrhs < 1) return h ? fail(h->gauge->ctx, {AMAMG_ERR_INVALID_ARG, "bad argument"}) : AMAMG_ERR_INVALID_ARG;
  amamg_context* ctx = h->gauge->ctx;
  try {
    REQUIRE(precision == AMAMG_FP64 || precision == AMAMG_MIXED_FP32, AMAMG_ERR_INVALID_ARG,
            "precision must be FP64 or MIXED_FP32");
    REQUIRE(level >= 0 && level + 1 < int(h->lv.size()), AMAMG_ERR_INVALID_ARG,
            "level must have a coarser level");
    REQUIRE(sweeps >= 1 && sweeps <= 16, AMAMG_ERR_INVALID_ARG, "sweeps must be in [1, 16]");
    HIPCHECK(hipSetDevice(ctx->device));
    amamg_gauge* gg = h->gauge;
    const LevelData& L = h->lv[level];
    const Geom& g = L.g;
    const int64_t nd = g.ndof();
    const bool f64 = precision == AMAMG_FP64;
    const Real T = f64 ? F64 : F32;
    const size_t cs = f64 ? sizeof(double2) : sizeof(float2);
    hipStream_t s = ctx->stream;
    Arena io;
    const size_t nval = size_t(nrhs) * nd;
    // x in the level's precision; f as the V-cycle holds it (FP64 on the fine level, whose
    // right-hand side is the Krylov vector, the level's precision below)
    auto upload = [&](const double* src, bool as64) -> void* {
      if (as64) {
        void* d = io.alloc<double2>(nval);
        HIPCHECK(hipMemcpyAsync(d, src, sizeof(double2) * nval, hipMemcpyHostToDevice, s));
        HIPCHECK(hipStreamSynchronize(s));
        return d;
      }
      std::vector<float2> h32(nval);
      for (size_t i = 0; i < nval; ++i) h32[i] = make_float2(float(src[2 * i]), float(src[2 * i + 1]));
      void* d = io.alloc<float2>(nval);
      HIPCHECK(hipMemcpyAsync(d, h32.data(), sizeof(float2) * nval, hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));
      return d;
    };
    void* dx = upload(x, f64);
    void* df = upload(f, f64 || level == 0);
    if (level == 0) {
      const LinkStore ls = f64 ? LINK_F64 : LINK_F32;
      ensure_links(gg, ls);
      void* dy = io.alloc<char>(cs * nval);
      wilson_gs_sweeps(s, ls, link0(gg, ls), link1(gg, ls), T, dx, dy, (const double2*)df, g.Lt, g.Lx, h->m0,
                       sweeps, nrhs, nd, nullptr);
      dx = dy;
    } else {
      const void* Ak = f64 ? (const void*)L.A : (const void*)L.A32;
      const void* Dk = f64 ? (const void*)L.Dinv : (const void*)L.Dinv32;
      for (int sw = 0; sw < sweeps; ++sw)
        for (int qb = 0; qb < 4; ++qb)
          stencil_gs_block(s, T, Ak, Dk, dx, df, g.Lt, g.Lx, g.b, qb, nrhs, nd, nullptr, 0, h->prm.block_smoother);
    }
    check_launch();
    if (f64) {
      HIPCHECK(hipMemcpyAsync(x, dx, sizeof(double2) * nval, hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
    } else {
      std::vector<float2> o32(nval);
      HIPCHECK(hipMemcpyAsync(o32.data(), dx, sizeof(float2) * nval, hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      for (size_t i = 0; i < nval; ++i) { x[2 * i] = o32[i].x; x[2 * i + 1] = o32[i].y; }
    }
  } catch (const Fail& f) {
    return fail(ctx, f);
  }
  return AMAMG_OK;
}

amamg_status amamg_get_test_vectors(const amamg_hierarchy* h, int32_t level, double* out) {
  if (!h || !out || level < 0 || level >= int(h->lv.size()) - 1) return AMAMG_ERR_INVALID_ARG;
  const LevelData& L = h->lv[level];
  if (!L.tv) return fail(h->gauge->ctx, {AMAMG_ERR_INVALID_ARG, "no test vectors (normalisation is not TESTVEC)"});
  return copy_out(h, out, L.tv, sizeof(double2) * h->prm.n_test_vectors * L.g.ndof());
}

}  // extern "C"
