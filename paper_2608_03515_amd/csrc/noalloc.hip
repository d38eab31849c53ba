// Transfers between two levels of a hierarchy on caller-owned device buffers, with no device
// allocation: the restriction's per-wirebasket partial sums (its only buffer beyond the input
// and the output) live in a fixed array of this translation unit, one copy per GPU, held until
// the process ends.  For callers that cannot call hipMalloc: code under HIP graph capture,
// tight serving loops, harnesses that forbid it.
//
// The kernels are those of amamg_apply_transfer and of the V-cycle (restriction P^H and
// prolongation P of the Multilevel approach), so the results are bitwise the same.  Every
// launch of the restriction writes every partial it later sums, so nothing in the array has
// to start at zero; calls that overlap on one GPU (several contexts or streams at once) share
// the array and race.
#include "runtime.hpp"

namespace amamg {
namespace rt {

constexpr size_t kScratchBytes = size_t(AMAMG_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) char scratch[kScratchBytes];

// Device address of each GPU's copy of `scratch`, looked up once per device with that device
// current.  In host code the array's name is only a host-side stand-in: kernels and copies get
// these addresses.
constexpr int kMaxDevices = 64;
static std::mutex scratch_mu;
static void* scratch_dev[kMaxDevices] = {};

void noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return;      // the entry point then reports it
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (scratch_dev[device]) return;
  void* p = nullptr;
  HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  scratch_dev[device] = p;
}

static void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(scratch_mu);
  return scratch_dev[device];
}

}  // namespace rt
}  // namespace amamg

using namespace amamg;
using namespace amamg::rt;

extern "C" amamg_status amamg_apply_transfer_noalloc(amamg_hierarchy* h, int32_t level, int32_t precision,
                                                     int32_t direction, int32_t nrhs, const void* in_dev,
                                                     void* out_dev) {
  if (!h) return AMAMG_ERR_INVALID_ARG;
  amamg_context* ctx = h->gauge->ctx;
  try {
    REQUIRE(in_dev && out_dev && nrhs >= 1, AMAMG_ERR_INVALID_ARG, "null device pointer or nrhs < 1");
    REQUIRE(aligned16(in_dev) && aligned16(out_dev), AMAMG_ERR_INVALID_ARG,
            "device pointers must be 16-byte aligned");
    REQUIRE(precision == AMAMG_FP64 || precision == AMAMG_MIXED_FP32, AMAMG_ERR_INVALID_ARG,
            "precision must be FP64 or MIXED_FP32");
    REQUIRE(level >= 0 && level + 1 < int(h->lv.size()), AMAMG_ERR_INVALID_ARG, "level must have a coarser level");
    REQUIRE(direction == 0 || direction == 1, AMAMG_ERR_INVALID_ARG, "direction must be 0 or 1");
    HIPCHECK(hipSetDevice(ctx->device));
    void* part = scratch_of(ctx->device);
    REQUIRE(part, AMAMG_ERR_DEVICE, "no scratch array on this device");
    const LevelData& L = h->lv[level];
    const Geom& g = L.g;
    const int64_t nd = g.ndof(), ndc = h->lv[level + 1].g.ndof();
    const bool f64 = precision == AMAMG_FP64;
    const Real T = f64 ? F64 : F32;
    const void* P = f64 ? (const void*)L.P : (const void*)L.P32;
    hipStream_t s = ctx->stream;
    if (direction == 0) {
      // the partial sums the restriction writes: [nrhs][wirebasket][chunk][column] in T
      const size_t cs = f64 ? sizeof(double2) : sizeof(float2);
      const size_t need = cs * size_t(nrhs) * size_t(g.nI) * g.nJ * size_t(restrict_chunks(g, L.nf, T)) * g.ncol();
      REQUIRE(need <= kScratchBytes, AMAMG_ERR_INVALID_ARG,
              "the restriction of " + std::to_string(nrhs) + " right-hand sides on level " + std::to_string(level) +
                  " needs " + std::to_string(need) + " bytes of partial sums; the fixed scratch array holds " +
                  std::to_string(kScratchBytes) + ": split the right-hand sides over several calls");
      restrict_(s, T, P, L.rows, L.nrows, L.nf, F64, in_dev, out_dev, part, g, nrhs, nd, ndc, nullptr);
    } else {
      prolong(s, T, P, L.rows, L.nrows, L.nf, in_dev, out_dev, g, 0, nrhs, nd, ndc, nullptr);
    }
    check_launch();
  } catch (const Fail& f) {
    return fail(ctx, f);
  }
  return AMAMG_OK;
}
