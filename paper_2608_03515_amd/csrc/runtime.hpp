// Host runtime of the AM-AMG library: handle types, device memory, the setup pipeline, the
// batched FGMRES driver and the request server.  Shared by the host translation units
// (runtime.hip: handles, setup and the C ABI; solve.hip: V-cycle and FGMRES driver;
// server.hip: continuous-batching server).
#pragma once

#include <array>
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/amamg.h"
#include "launch.hpp"

namespace amamg {
namespace rt {

struct Fail {
  amamg_status code;
  std::string msg;
};

#define HIPCHECK(expr)                                                                          \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) {                                                                     \
      if (e_ == hipErrorOutOfMemory)                                                            \
        throw ::amamg::rt::Fail{AMAMG_ERR_OUT_OF_MEMORY, std::string(#expr) + ": out of device memory"}; \
      throw ::amamg::rt::Fail{AMAMG_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    }                                                                                           \
  } while (0)

#define REQUIRE(cond, code, msg)                        \
  do {                                                  \
    if (!(cond)) throw ::amamg::rt::Fail{code, msg};    \
  } while (0)

// Device allocations owned by a handle, released together; `bytes` counts what is held.
struct Arena {
  std::vector<void*> ptrs;
  size_t bytes = 0;
  template <typename T> T* alloc(size_t count) {
    if (count == 0) count = 1;
    void* p = nullptr;
    HIPCHECK(hipMalloc(&p, count * sizeof(T)));
    ptrs.push_back(p);
    bytes += count * sizeof(T);
    return static_cast<T*>(p);
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
  }
  Arena() = default;
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  ~Arena() { release(); }
};

// Device buffers looked up by (name, level): allocated on first use, reused afterwards, so a
// repeated setup on the same hierarchy allocates nothing.
struct Pool {
  struct Item { std::string key; void* p; size_t bytes; };
  std::vector<Item> items;
  template <typename T> T* get(const char* name, int level, size_t count) {
    if (count == 0) count = 1;
    const std::string key = std::string(name) + "#" + std::to_string(level);
    for (Item& it : items)
      if (it.key == key) {
        if (it.bytes >= count * sizeof(T)) return static_cast<T*>(it.p);
        (void)hipFree(it.p);
        it.p = nullptr;
        HIPCHECK(hipMalloc(&it.p, count * sizeof(T)));
        it.bytes = count * sizeof(T);
        return static_cast<T*>(it.p);
      }
    void* p = nullptr;
    HIPCHECK(hipMalloc(&p, count * sizeof(T)));
    items.push_back({key, p, count * sizeof(T)});
    return static_cast<T*>(p);
  }
  size_t bytes() const {
    size_t s = 0;
    for (const Item& it : items) s += it.bytes;
    return s;
  }
  Pool() = default;
  Pool(const Pool&) = delete;
  Pool& operator=(const Pool&) = delete;
  ~Pool() {
    for (Item& it : items) (void)hipFree(it.p);
  }
};

// Benchmark timer: HIP events around every launch of one kernel family in the solve.  A
// launch's algorithmic bytes are its per-rhs bytes (the fields it reads and writes) times the
// right-hand sides it served, which the host learns at the end of each restart cycle of the
// batch (group) that ran it, plus its per-launch bytes (operators every right-hand side shares:
// links, interpolation weights, coarse blocks), counted once.
// Launch-shape autotuner for kernels whose arithmetic does not depend on the launch shape (the
// results are bitwise the same for every candidate).  Entries are keyed by what decides the best
// shape: the tunable, the grid, block size, precision and batch size.
struct Tuner {
  enum Kind { FINE_GS_TILE = 0, COARSE_GS_RHS = 1 };
  struct Entry {
    int choice = 0;                  // the chosen candidate value
    std::vector<int> cand;           // candidate values
    std::vector<double> us;          // their measured times (empty when not timed)
  };
  std::mutex mu;
  int mode = 0;                      // amamg_tune_mode
  int force = 0;
  std::map<std::array<int, 6>, Entry> entries;   // {kind, lt, lx, b, precision, nrhs}
};

struct KernelTimer {
  static constexpr int NF = 8;
  uint32_t mask = 0;
  std::vector<hipEvent_t> events;
  struct Rec { int e0, e1, step, family, group; double bytes_per_rhs, bytes_per_launch; };
  std::vector<Rec> pending;
  int64_t launches[NF] = {};
  double total_ms[NF] = {}, total_bytes[NF] = {};
};

struct LevelData {
  Geom g{};
  bool coarsest = false;
  // operator of this level (k >= 1)
  double2* A = nullptr;      // stencil [nnode][25][b][b] (non-coarsest)
  float2* A32 = nullptr;
  double2* Dinv = nullptr;   // [nnode][b][b]
  float2* Dinv32 = nullptr;
  double2* Adense = nullptr; // coarsest [n][n]
  double2* Ainv = nullptr;   // coarsest inverse [n][n]
  double2* Acm = nullptr;    // coarsest matrix, column-major [k][row] (GMRES variant only)
  double2* G = nullptr;      // mass term: G_k = P^H G_{k-1} P, G_0 = I (stencil, or dense at the
                             // coarsest; made by the first mass shift)
  // transfer to the next level (non-coarsest)
  int8_t* kind = nullptr;
  int* owner = nullptr;
  int* node = nullptr;
  double2* P = nullptr;      // [nnode][b][4 bc]
  float2* P32 = nullptr;
  double2* tv = nullptr;     // smoothed test vectors [nv][ndof]
  int* tabs = nullptr;       // footprint tables: postab [fp] then fpos [nf]
  int nf = 0;                // F positions per wirebasket footprint
  int* rows = nullptr;       // owned fine rows per wirebasket [nW][nf*b]
  int* nrows = nullptr;      // their counts [nW]
};

// Everything a running batched solve writes: Krylov basis and search directions, Hessenberg
// and Givens data, per-rhs control state and residual history, the V-cycle's per-level
// vectors, and pinned host mirrors of the state.  `cap` right-hand-side slots.
struct Workspace {
  int cap = 0, m = 0, hist_cap = 0;
  Real prec = F64;
  std::vector<int64_t> shape;   // per-level unknowns and restriction partial counts it was sized for
  // device buffers are carved from one block that only grows, so rebinding a workspace to
  // another hierarchy frees nothing (hipFree would wait for the whole device)
  void* block = nullptr;
  size_t block_bytes = 0;
  int host_cap = 0, host_hist = 0;   // sizes of the pinned mirrors
  double2 *V = nullptr, *w = nullptr, *H = nullptr, *g = nullptr, *sn = nullptr, *y = nullptr;
  double2 *part = nullptr, *hist = nullptr;
  double2* coef = nullptr;    // Gram update coefficients [cap][64]
  double* cs = nullptr;
  double* zsc = nullptr;      // search-direction scales 1 / rho_j [cap][m]
  void* Z = nullptr;
  RhsState* st = nullptr;     // control state of the running batch
  RhsState* st2 = nullptr;    // state of slots being admitted
  int* admit = nullptr;       // admission mask [cap]
  struct Lev { void *f = nullptr, *x = nullptr, *tmp = nullptr, *rpart = nullptr; double2* kry = nullptr; };
  std::vector<Lev> lv;
  RhsState* hst = nullptr;    // pinned mirrors
  RhsState* hst2 = nullptr;
  int* hadmit = nullptr;
  double2* hhist = nullptr;
  hipEvent_t ev = nullptr;
  // restart cycle captured into a HIP graph (solve param `graphs`) and the launch it was
  // captured for: every pointer and value the kernels receive; replayed while that matches
  hipGraphExec_t graph = nullptr;
  std::vector<uint64_t> graph_key;
  Workspace() = default;
  Workspace(const Workspace&) = delete;
  Workspace& operator=(const Workspace&) = delete;
  ~Workspace();
  void release();
};

}  // namespace rt
}  // namespace amamg

struct amamg_context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  amamg::rt::KernelTimer timer;
  amamg::rt::Tuner tuner;
};

struct amamg_gauge {
  amamg_context* ctx = nullptr;
  int nt = 0, nx = 0;
  double m0 = 0;
  int nhier = 0;
  amamg::rt::Arena mem;
  double2* U = nullptr;     // [2][nt*nx]
  float2* U32 = nullptr;
  amamg::bf16c* U16 = nullptr;
  int version = 0;          // bumped by amamg_gauge_update_links
  int v32 = -1, v16 = -1;   // version the low-precision copies were made from
};

struct amamg_hierarchy {
  amamg_gauge* gauge = nullptr;
  amamg_setup_params prm{};
  double m0 = 0;
  std::vector<amamg::rt::LevelData> lv;
  amamg::rt::Pool mem;      // setup products and setup scratch
  // workspaces and extra streams of the plain solve calls (one per right-hand-side group)
  std::vector<amamg::rt::Workspace*> ws;
  std::vector<hipStream_t> streams;
  std::vector<std::vector<double2>> history;
  uint64_t generation = 0;  // number of its last setup or mass shift, unique in the process
                            // (graphs key on it)
  bool mass_terms = false;  // LevelData::G of every coarse level is current
  // A derived hierarchy (derive_mass) shares its base's wirebaskets, interpolation and mass
  // terms and owns only its operators; the base counts its derived hierarchies and may not be
  // set up again, moved or destroyed while any exists.
  amamg_hierarchy* base = nullptr;
  int derived = 0;
  ~amamg_hierarchy();
};

namespace amamg {
namespace rt {

amamg_status fail(amamg_context* ctx, const Fail& f);
// device address of the no-allocation scratch array on `device` (current), looked up once
void noalloc_init(int device);
bool aligned16(const void* p);
void check_launch();
bool finite_all(const double* v, size_t n);

// kernel timer (the family's events are recorded on the stream `s` of the launch)
int timer_start(amamg_context* ctx, hipStream_t s, int family, int step, int group, double bytes_per_rhs,
                double bytes_per_launch = 0.0);
void timer_stop(amamg_context* ctx, hipStream_t s, int rec);

// setup with the hierarchy's mass h->m0, synchronous on `stream` (null: the context stream);
// with `scratch`, the setup's temporary buffers come from that pool (kept for the next setup)
// and the hierarchy holds only what the solve uses
void run_setup(amamg_hierarchy* h, hipStream_t stream = nullptr, Pool* scratch = nullptr);
// moves a built hierarchy to bare mass m0, keeping its wirebaskets, test vectors and
// interpolation (A_k += (m0 - m0_old) G_k on every coarse level, then the smoother blocks, the
// coarsest inverse and the FP32 copies again); synchronous on `stream` (null: context stream)
void shift_mass(amamg_hierarchy* h, double m0, hipStream_t stream = nullptr);
uint64_t next_generation();
// the mass terms G_k of every coarse level (once per setup; shift_mass calls it too)
void ensure_mass_terms(amamg_hierarchy* h, hipStream_t stream = nullptr);
// a new hierarchy at bare mass m0 that shares base's wirebaskets, interpolation and mass terms
// and owns its operators, smoother blocks and coarsest inverse; synchronous on `stream`.  base
// must have its mass terms (ensure_mass_terms) and is only read; the caller adds the result to
// base->derived and gauge->nhier.
amamg_hierarchy* derive_mass(amamg_hierarchy* base, double m0, hipStream_t stream = nullptr);
// device bytes a hierarchy derived from h holds (its operators, smoother blocks, coarsest
// inverse and FP32 copies) plus the temporaries of its factorisations
size_t derive_bytes(const amamg_hierarchy* h);
// device bytes a hierarchy of these parameters holds after setup (estimate, for admission)
size_t setup_bytes(int nt, int nx, const amamg_setup_params& p);

// low-precision link copies of a gauge (made on the context stream, once per link version)
void ensure_links(amamg_gauge* gg, LinkStore ls);
const void* link0(amamg_gauge* g, LinkStore ls);
const void* link1(amamg_gauge* g, LinkStore ls);

// workspaces
// (Re)allocate unless the workspace was sized for exactly this hierarchy shape, slot count,
// restart length and precision (and at least this history length).
void ensure_workspace(Workspace& ws, const amamg_hierarchy* h, int cap, int m, Real prec, int hist_cap);
bool workspace_fits(const Workspace& ws, const amamg_hierarchy* h, int cap, int m, Real prec, int hist_cap);
size_t workspace_bytes(const amamg_hierarchy* h, int cap, int m, Real prec, int hist_cap);

// One batched FGMRES run over a workspace on one stream, driven from the host in steps:
// admission of slots (two host round trips: the input check, then the first cycle start),
// then one restart cycle per step.  The host never blocks inside: after every enqueued stage
// it records the workspace event and waits for `ready()`.
struct Batch {
  amamg_hierarchy* h = nullptr;
  Workspace* ws = nullptr;
  hipStream_t s = nullptr;
  amamg_solve_params p{};
  int group = 0;                // kernel-timer group
  const double2* b = nullptr;   // [cap][n] right-hand sides
  double2* x = nullptr;         // [cap][n] iterates
  // host view
  std::vector<int> cycle_in;    // slots in the cycle that was enqueued last
  std::vector<int> pending;     // slots whose admission awaits the input check
  bool cycle_enqueued = false;
  // launch shapes from the context's tuner: fine smoother tile width, right-hand sides per
  // wave of each level's paired block smoother (0 = default)
  int fine_tc = 0;
  std::vector<int> gs_rb;

  void init(amamg_hierarchy* h, Workspace* ws, hipStream_t s, const amamg_solve_params& p,
            const double2* b, double2* x, int group);
  // enqueue the input check of `slots` (||b||, non-finite and zero right-hand sides)
  void admit_begin(const std::vector<int>& slots);
  // after ready(): slots of the pending admission whose input is non-finite
  std::vector<int> admit_nonfinite() const;
  // enqueue the first cycle start of the pending slots except `reject` (x = 0 unless the
  // initial guess is used, r = b - D x, V_0 = r / ||r||) and merge them into the batch state
  void admit_finish(const std::vector<int>& reject, bool use_initial_guess);
  // enqueue one restart cycle for every slot in a cycle (requires a state read first); with
  // p.graphs the cycle is captured into a HIP graph on first use and replayed
  void enqueue_cycle();
  void enqueue_cycle_kernels();
  // the cycle's pieces: step j's V-cycle and matvec, step j's Gram-Schmidt, the cycle's end
  void enqueue_step_front(int j);
  void enqueue_step_krylov(int j);
  void enqueue_cycle_tail();
  KrylovSeg krylov_seg() const;
  // enqueue a copy of the state to the pinned mirror and record the event
  void enqueue_state_read();
  bool ready() const;
  // after ready(): host copy of the batch state (valid after enqueue_state_read)
  const RhsState& state(int slot) const { return ws->hst[slot]; }
  // after a state read: flush the kernel timer and note which slots are in the next cycle;
  // returns true when some slot is in a cycle
  bool cycle_boundary();
  // residual history of a slot (synchronous copy on the batch stream)
  std::vector<double2> history(int slot) const;
};

// plain solve of nrhs right-hand sides (caller's device buffers), split into `groups`
// batches on separate streams
amamg_status run_solve(amamg_hierarchy* h, int nrhs, const double2* b, double2* x,
                       const amamg_solve_params& p, amamg_solve_info* info);
// several lattices (distinct hierarchies of one context) in lock step, the Gram-Schmidt of
// each step in one launch for all of them; after `root`'s queued work, which then follows the
// solve; blocks until the solve has finished
amamg_status run_solve_multi(const std::vector<amamg_hierarchy*>& hs, const std::vector<int>& nrhs,
                             const std::vector<const double2*>& b, const std::vector<double2*>& x,
                             const amamg_solve_params& p, amamg_solve_info* info, hipStream_t root);

}  // namespace rt
}  // namespace amamg
