// Shared device helpers and internal declarations of the AM-AMG HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace amamg {

// ------------------------------------------------------------------ complex arithmetic

template <typename R> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename R> using cplx = typename cvec<R>::type;

template <typename R> __device__ __host__ inline cplx<R> mk(R re, R im) { cplx<R> z; z.x = re; z.y = im; return z; }
template <typename R> __device__ __host__ inline cplx<R> czero() { return mk<R>(R(0), R(0)); }
template <typename V> __device__ __host__ inline V cadd(V a, V b) { V z; z.x = a.x + b.x; z.y = a.y + b.y; return z; }
template <typename V> __device__ __host__ inline V csub(V a, V b) { V z; z.x = a.x - b.x; z.y = a.y - b.y; return z; }
template <typename V> __device__ __host__ inline V cmul(V a, V b) {
  V z; z.x = a.x * b.x - a.y * b.y; z.y = a.x * b.y + a.y * b.x; return z;
}
// conj(a) * b
template <typename V> __device__ __host__ inline V cmulc(V a, V b) {
  V z; z.x = a.x * b.x + a.y * b.y; z.y = a.x * b.y - a.y * b.x; return z;
}
// acc + a * b
template <typename V> __device__ __host__ inline V cfma(V a, V b, V acc) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
  return acc;
}
// acc + conj(a) * b
template <typename V> __device__ __host__ inline V cfmac(V a, V b, V acc) {
  acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
  return acc;
}
template <typename V, typename R> __device__ __host__ inline V cscale(V a, R s) { V z; z.x = a.x * s; z.y = a.y * s; return z; }
template <typename V> __device__ __host__ inline V cconj(V a) { V z; z.x = a.x; z.y = -a.y; return z; }
// a / b = a conj(b) / |b|^2
template <typename V> __device__ __host__ inline V cdiv(V a, V b) {
  const auto d = 1 / (b.x * b.x + b.y * b.y);
  V z; z.x = (a.x * b.x + a.y * b.y) * d; z.y = (a.y * b.x - a.x * b.y) * d; return z;
}
template <typename V> __device__ __host__ inline V ctimes_i(V a) { V z; z.x = -a.y; z.y = a.x; return z; }
template <typename V> __device__ __host__ inline auto cabs2(V a) { return a.x * a.x + a.y * a.y; }

// conversions between storage types
template <typename To, typename From> __device__ __host__ inline To cconv(From a) { To z; z.x = a.x; z.y = a.y; return z; }

// BF16-stored link: two bfloat16 (re, im) packed in 32 bits
struct bf16c { uint32_t bits; };

__device__ __host__ inline float bf16_to_f32(uint16_t h) {
  union { uint32_t u; float f; } v; v.u = uint32_t(h) << 16; return v.f;
}
__device__ __host__ inline uint16_t f32_to_bf16_rne(float f) {
  union { uint32_t u; float f; } v; v.f = f;
  uint32_t u = v.u;
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return uint16_t(u >> 16);
}

// link loads: FP64, FP32 or BF16 storage, returned in compute type R
template <typename R, typename L> __device__ inline cplx<R> load_link(const L* U, int64_t i);
template <> __device__ inline double2 load_link<double, double2>(const double2* U, int64_t i) { return U[i]; }
template <> __device__ inline float2 load_link<float, float2>(const float2* U, int64_t i) { return U[i]; }
template <> __device__ inline float2 load_link<float, bf16c>(const bf16c* U, int64_t i) {
  uint32_t b = U[i].bits;
  return make_float2(bf16_to_f32(uint16_t(b & 0xFFFFu)), bf16_to_f32(uint16_t(b >> 16)));
}

// ------------------------------------------------------------------------- utilities

#define AMAMG_WAVE 64

// XCD-aware block order: gfx950 dispatches consecutive workgroups round-robin over its 8
// XCDs, each with its own L2.  Remap so that each XCD works on a contiguous range of tiles
// (neighbouring lattice rows then meet in the same L2).
__device__ inline int xcd_block(int bid, int nblk) {
  const int nx = 8;
  if (nblk < 2 * nx) return bid;
  int per = nblk / nx, rem = nblk % nx;
  int x = bid % nx, k = bid / nx;
  // XCD x receives blocks x, x+8, ...: give it tiles [start_x, start_x + count_x)
  int start = x * per + (x < rem ? x : rem);
  int count = per + (x < rem ? 1 : 0);
  return k < count ? start + k : bid;   // k < count always holds for a full grid
}

template <typename T> __device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = AMAMG_WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Sweep order of the 16 coarse colours c = (I mod 4) 4 + (J mod 4): the four colours of each
// 2 x 2 block of the colour pattern in a row.  Block qb (0..3) holds (a, 2q), (a, 2q + 1),
// (a + 1, 2q), (a + 1, 2q + 1) with a = 2 (qb >> 1), q = qb & 1.
__host__ __device__ constexpr int coarse_colour(int i) {
  return 4 * (2 * ((i >> 2) >> 1) + ((i >> 1) & 1)) + 2 * ((i >> 2) & 1) + (i & 1);
}

// Global-to-LDS staging with U loads in flight per thread.  For every index q < total (thread
// t takes q = t, t + NT, ...), fetch(q) is issued for U indices before store(q, value) runs for
// them.  A plain loop of load-then-store lets each load wait for the previous iteration's LDS
// store (the next address often comes from LDS too), one memory round trip per element; here one
// round trip covers U elements.  fetch must only load (no arithmetic on the loaded value, which
// would wait for it) and runs unconditionally, for indices past the end clamped to total - 1, so
// that no branch separates the loads; the stores are guarded.  Call with all NT threads.
template <int U, int NT, typename T, typename Fetch, typename Store>
__device__ inline void stage(int total, Fetch fetch, Store store) {
  for (int q0 = int(threadIdx.x); q0 < total; q0 += NT * U) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + NT * u;
      v[u] = fetch(q < total ? q : total - 1);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + NT * u;
      if (q < total) store(q, v[u]);
    }
  }
}

// ------------------------------------------------------------------ device structures

// Per right-hand-side FGMRES state (device resident).
struct RhsState {
  double bnorm;       // ||b||
  double beta;        // ||r|| at cycle start
  double inv_h;       // 1 / h_{j+1,j} of the last step
  double true_res;    // last true relative residual
  double est;         // last |g_{j+1}| / ||b||
  int active;         // still iterating in the current cycle
  int in_cycle;       // took part in the current cycle
  int k;              // Arnoldi steps in the current cycle
  int iters;          // Arnoldi steps in total
  int restarts;
  int converged;
  int done;           // finished: converged or capped
  int hist_len;
  int nonfinite;
  int last_k;         // Arnoldi steps of the cycle that ended last
  int pad;
};

}  // namespace amamg
