// FGMRES(m) kernels, FP64 (paper: FGMRES outer solver, relative tolerance 1e-10).
//
// Right-preconditioned flexible Arnoldi with classical Gram-Schmidt applied twice.  Every
// reduction is two-level and fixed-order: each block writes its partial sums, and the block
// that finishes last (a device-scope counter decides which) adds the partials in block
// order.  Results are therefore bitwise reproducible although blocks finish in any order.
// The last block also runs the scalar bookkeeping that needs the reduced value (Hessenberg
// column, Givens rotations, cycle start and end), so no extra launch is spent on it.
//
// Givens rotation for (a, b) = (H_jj, H_{j+1,j}): nu = sqrt(|a|^2 + |b|^2), c = |a| / nu,
// s = (a / |a|) conj(b) / nu (c = 0, s = 1 when a = 0); a rotation maps (x, y) to
// (c x + s y, -conj(s) x + c y); g_{j+1} = -conj(s) g_j, g_j = c g_j.
//
// Vector layouts: basis V [j][rhs][n], search directions Z [j][rhs][n], w and x [rhs][n].
#include <array>
#include <utility>

#include "launch.hpp"

namespace amamg {

#define KMAXV 32

template <int NV>
__device__ inline void block_partial(const double2 (&acc)[NV], int nv, double2* out, double* lds) {
  // lds: NV * 4 * 2 doubles; writes nv block totals to out[0..nv)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if (i < nv) {
      const double re = wave_sum(acc[i].x), im = wave_sum(acc[i].y);
      if (lane == 0) { lds[(i * 4 + wv) * 2] = re; lds[(i * 4 + wv) * 2 + 1] = im; }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
    double re = 0, im = 0;
    for (int q = 0; q < 4; ++q) { re += lds[(i * 4 + q) * 2]; im += lds[(i * 4 + q) * 2 + 1]; }
    out[i] = make_double2(re, im);
  }
}

// fin[i] = sum over blocks of part_r[blk][i] for i < nv, added in a fixed order (8 strided
// groups of blocks with eight independent partial sums each, then the groups in order).  Every
// kernel that needs the total recomputes it with this routine, so all agree bitwise.  Must be
// called by all 256 threads; fin and scratch are shared arrays.
__device__ inline void sum_blocks(const double2* __restrict__ part_r, int nblk, int nv,
                                  double2* fin, double2* scratch) {
  const int i = threadIdx.x & (KMAXV - 1), c = threadIdx.x / KMAXV;
  double2 s = make_double2(0, 0);
  if (i < nv) {
    double2 q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) q[u] = make_double2(0, 0);
    for (int b = c; b < nblk; b += 64) {
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (b + 8 * u < nblk) q[u] = cadd(q[u], part_r[int64_t(b + 8 * u) * KMAXV + i]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s = cadd(s, q[u]);
  }
  scratch[c * KMAXV + i] = s;
  __syncthreads();
  if (threadIdx.x < nv) {
    double2 t = make_double2(0, 0);
    for (int q = 0; q < 8; ++q) t = cadd(t, scratch[q * KMAXV + threadIdx.x]);
    fin[threadIdx.x] = t;
  }
  __syncthreads();
}

__device__ inline bool finite_d(double v) { return v == v && v - v == 0.0; }

struct ArnoldiArgs {
  double2* H;       // [rhs][(m+1) m], H[i][j] at i*m + j
  double* cs;       // [rhs][m]
  double2* sn;      // [rhs][m]
  double2* g;       // [rhs][m+1]
  int j;
  double tol, inner_tol;
  int max_iters;
  double2* hist;
  int hist_cap;
};

// Arnoldi step j for one rhs, given hn = ||w|| after CGS2: col[0..j] = h1 + h2 is the new
// Hessenberg column and col[j + 1] = hn; the earlier rotations csl/snl (all in LDS).  Rotates
// the column, forms rotation j and updates g; the caller writes the column back to H.
__device__ inline void arnoldi_step(const KrylovDims& dm, RhsState& s, int r, double hn, double2* col,
                                    const double* csl, const double2* snl, const ArnoldiArgs& a) {
  const int m = dm.m, j = a.j;
  double* csr = a.cs + int64_t(r) * m;
  double2* snr = a.sn + int64_t(r) * m;
  double2* gr = a.g + int64_t(r) * (m + 1);
  for (int i = 0; i < j; ++i) {
    const double2 x = col[i], y = col[i + 1];
    const double c = csl[i];
    const double2 sv = snl[i];
    col[i] = cadd(cscale(x, c), cmul(sv, y));
    col[i + 1] = csub(cscale(y, c), cmulc(sv, x));
  }
  const double2 av = col[j], bv = col[j + 1];
  double c;
  double2 sv;
  const double aa = sqrt(cabs2(av));
  if (aa == 0.0) {
    c = 0.0;
    sv = make_double2(1.0, 0.0);
  } else {
    const double nu = sqrt(cabs2(av) + cabs2(bv));
    c = aa / nu;
    sv = cscale(cmul(make_double2(av.x / aa, av.y / aa), cconj(bv)), 1.0 / nu);
  }
  col[j] = cadd(cscale(av, c), cmul(sv, bv));
  col[j + 1] = make_double2(0, 0);
  csr[j] = c;
  snr[j] = sv;
  const double2 gj = gr[j];
  gr[j + 1] = cscale(cmulc(sv, gj), -1.0);
  gr[j] = cscale(gj, c);
  s.iters += 1;
  s.k = j + 1;
  const double gabs = sqrt(cabs2(gr[j + 1]));
  s.est = gabs / s.bnorm;
  if (s.hist_len < a.hist_cap) a.hist[int64_t(r) * a.hist_cap + s.hist_len++] = make_double2(s.est, 0.0);
  bool end = (gabs <= a.tol * s.bnorm) || (hn <= 1e-300 * s.bnorm) || (s.iters >= a.max_iters) ||
             (j + 1 == m) || (a.inner_tol > 0.0 && gabs <= a.inner_tol * s.beta);
  if (!finite_d(hn) || !finite_d(gabs)) { s.nonfinite = 1; end = true; }
  if (end) s.active = 0;
  else s.inv_h = 1.0 / hn;
}

// partials of h = V^H w  (V_0 .. V_{NV-1}); NV is a compile-time count so the accumulators
// fit the actual basis size
template <int NV>
__global__ __launch_bounds__(256) void k_dots(KrylovDims dm, const double2* __restrict__ V,
                                              int64_t vsj, const double2* __restrict__ w,
                                              double2* __restrict__ part,
                                              const RhsState* __restrict__ st) {
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  __shared__ double lds[2 * NV * 4];
  double2 acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = make_double2(0, 0);
  const double2* wr = w + r * dm.n;
  const double2* Vr = V + r * dm.n;
  for (int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x; d < dm.n; d += int64_t(gridDim.x) * 256) {
    const double2 wd = wr[d];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = cfmac(Vr[i * vsj + d], wd, acc[i]);
  }
  block_partial<NV>(acc, NV, part + (int64_t(r) * gridDim.x + blockIdx.x) * KMAXV, lds);
}

// w -= sum_i V_i h_i with h the total of the previous kernel's partials hpart; then partials
// of ||w_new||^2 into part.
template <int NV>
__global__ __launch_bounds__(256) void k_update_norm(KrylovDims dm, const double2* __restrict__ V,
                                                     int64_t vsj, double2* __restrict__ w,
                                                     const double2* __restrict__ hpart,
                                                     double2* __restrict__ part,
                                                     const RhsState* __restrict__ st) {
  const int r = blockIdx.y;
  if (!st[r].active) return;
  __shared__ double lds[2 * 4];
  __shared__ double2 hs[KMAXV], scratch[8 * KMAXV];
  sum_blocks(hpart + int64_t(r) * gridDim.x * KMAXV, gridDim.x, NV, hs, scratch);
  double2 acc[1] = {make_double2(0, 0)};
  double2* wr = w + r * dm.n;
  const double2* Vr = V + r * dm.n;
#pragma unroll 1
  for (int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x; d < dm.n; d += int64_t(gridDim.x) * 256) {
    double2 wd = wr[d];
#pragma unroll
    for (int i = 0; i < NV; ++i) wd = csub(wd, cmul(Vr[i * vsj + d], hs[i]));
    wr[d] = wd;
    acc[0].x += cabs2(wd);
  }
  block_partial<1>(acc, 1, part + (int64_t(r) * gridDim.x + blockIdx.x) * KMAXV, lds);
}

// Lanes per element of the fused update: enough to keep the per-lane share of the basis (and
// its accumulators) in a few registers, few enough that the shuffles stay cheap.
constexpr int update_lanes(int nv) { return nv <= 2 ? 1 : nv <= 12 ? 2 : 4; }

// Fused first-projection update and second projection: w -= sum_i V_i h_i (h from hpart), then
// partials of V^H w_new into part, in one pass over V.  S lanes share an element: lane `sub`
// holds the basis vectors i = sub + S k in registers, the S partial sums of V_i h_i are added
// with lane shuffles, and every lane then accumulates conj(V_i) w_new for its own vectors, so
// each basis value is read from memory once.
template <int NV, int S>
__global__ __launch_bounds__(256) void k_update_dots(KrylovDims dm, const double2* __restrict__ V,
                                                     int64_t vsj, double2* __restrict__ w,
                                                     const double2* __restrict__ hpart,
                                                     double2* __restrict__ part,
                                                     const RhsState* __restrict__ st) {
  constexpr int K = (NV + S - 1) / S, EPB = 256 / S;
  const int r = blockIdx.y;
  if (!st[r].active) return;
  __shared__ double2 hs[KMAXV], scratch[8 * KMAXV], red[4][KMAXV];
  sum_blocks(hpart + int64_t(r) * gridDim.x * KMAXV, gridDim.x, NV, hs, scratch);
  const int sub = threadIdx.x % S;
  double2 hk[K], acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = sub + S * k;
    hk[k] = i < NV ? hs[i] : make_double2(0, 0);
    acc[k] = make_double2(0, 0);
  }
  double2* wr = w + r * dm.n;
  const double2* Vr = V + r * dm.n;
#pragma unroll 1
  for (int64_t d = int64_t(blockIdx.x) * EPB + threadIdx.x / S; d < dm.n; d += int64_t(gridDim.x) * EPB) {
    double2 v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = sub + S * k;
      v[k] = i < NV ? Vr[i * vsj + d] : make_double2(0, 0);
    }
    double2 p = make_double2(0, 0);
#pragma unroll
    for (int k = 0; k < K; ++k) p = cfma(v[k], hk[k], p);
#pragma unroll
    for (int o = 1; o < S; o <<= 1) {
      p.x += __shfl_xor(p.x, o);
      p.y += __shfl_xor(p.y, o);
    }
    const double2 wd = csub(wr[d], p);
    if (sub == 0) wr[d] = wd;
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = cfmac(v[k], wd, acc[k]);
  }
  // block totals: lanes with equal `sub` hold the same basis vectors (xor offsets S .. 32 within
  // a wave), then the four waves in order
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double2 a = acc[k];
#pragma unroll
    for (int o = S; o < 64; o <<= 1) {
      a.x += __shfl_xor(a.x, o);
      a.y += __shfl_xor(a.y, o);
    }
    const int i = sub + S * k;
    if (lane < S && i < NV) red[wv][i] = a;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double2 t = red[0][threadIdx.x];
    for (int q = 1; q < 4; ++q) t = cadd(t, red[q][threadIdx.x]);
    part[(int64_t(r) * gridDim.x + blockIdx.x) * KMAXV + threadIdx.x] = t;
  }
}

// Arnoldi step j, one block per rhs: h1, h2 and ||w||^2 are the totals of the three partial
// sets of the Gram-Schmidt kernels.
__global__ __launch_bounds__(256) void k_arnoldi(KrylovDims dm, const double2* __restrict__ p1,
                                                 const double2* __restrict__ p2,
                                                 const double2* __restrict__ p3,
                                                 RhsState* __restrict__ st, ArnoldiArgs aa, int nv) {
  const int r = blockIdx.x;
  if (!st[r].active) return;
  __shared__ double2 h1[KMAXV], h2[KMAXV], hn[KMAXV], scratch[8 * KMAXV];
  __shared__ double2 col[KMAXV + 1], snl[KMAXV];
  __shared__ double csl[KMAXV];
  sum_blocks(p1 + int64_t(r) * dm.nblk * KMAXV, dm.nblk, nv, h1, scratch);
  sum_blocks(p2 + int64_t(r) * dm.nblk * KMAXV, dm.nblk, nv, h2, scratch);
  sum_blocks(p3 + int64_t(r) * dm.nblk * KMAXV, dm.nblk, 1, hn, scratch);
  const int m = dm.m, j = aa.j;
  for (int i = threadIdx.x; i <= j; i += blockDim.x) col[i] = cadd(h1[i], h2[i]);
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    csl[i] = aa.cs[int64_t(r) * m + i];
    snl[i] = aa.sn[int64_t(r) * m + i];
  }
  if (threadIdx.x == 0) col[j + 1] = make_double2(sqrt(hn[0].x), 0.0);
  __syncthreads();
  if (threadIdx.x == 0) {
    RhsState s = st[r];
    arnoldi_step(dm, s, r, sqrt(hn[0].x), col, csl, snl, aa);
    st[r] = s;
  }
  __syncthreads();
  double2* Hr = aa.H + int64_t(r) * (m + 1) * m;
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) Hr[i * m + j] = col[i];
}

// ||x||^2 per rhs whose state is active, then: mode 1 fresh states (x = b; the host marks the
// slots to start as active); 2 first cycle start (x = r_0); 3 end of a cycle (x = b - D x):
// convergence test and the next cycle's start.
struct CycleArgs {
  double2* g;
  double tol;
  int max_iters;
  double2* hist;
  int hist_cap;
};

__device__ inline void begin_cycle(const KrylovDims& dm, RhsState& s, int r, double beta,
                                   int first, const CycleArgs& ca) {
  s.last_k = s.k;
  if (s.done || !s.in_cycle || s.nonfinite) {
    if (s.nonfinite) s.done = 1;
    s.active = 0;
    s.in_cycle = 0;
    return;
  }
  s.true_res = beta / s.bnorm;
  if (!finite_d(beta)) { s.nonfinite = 1; s.done = 1; s.active = 0; s.in_cycle = 0; return; }
  if (!first && s.hist_len < ca.hist_cap)
    ca.hist[int64_t(r) * ca.hist_cap + s.hist_len++] = make_double2(s.true_res, 1.0);
  if (beta <= ca.tol * s.bnorm) {
    s.converged = 1; s.done = 1; s.active = 0; s.in_cycle = 0;
  } else if (s.iters >= ca.max_iters) {
    s.done = 1; s.active = 0; s.in_cycle = 0;
  } else {
    if (!first) s.restarts += 1;
    s.beta = beta;
    s.inv_h = 1.0 / beta;
    s.k = 0;
    s.active = 1;
    s.in_cycle = 1;
    double2* gr = ca.g + int64_t(r) * (dm.m + 1);
    gr[0] = make_double2(beta, 0.0);
    for (int i = 1; i <= dm.m; ++i) gr[i] = make_double2(0, 0);
  }
}

__global__ __launch_bounds__(256) void k_norm(KrylovDims dm, const double2* __restrict__ x,
                                              double2* __restrict__ part,
                                              const RhsState* __restrict__ st) {
  const int r = blockIdx.y;
  if (!st[r].active) return;
  __shared__ double lds[2 * KMAXV * 4];
  double2 acc[1] = {make_double2(0, 0)};
  const double2* xr = x + r * dm.n;
  for (int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x; d < dm.n; d += int64_t(gridDim.x) * 256)
    acc[0].x += cabs2(xr[d]);
  block_partial<1>(acc, 1, part + (int64_t(r) * gridDim.x + blockIdx.x) * KMAXV, lds);
}

// one block per rhs: mode 1 fresh states (x = b); 2 first cycle start (x = r_0); 3 end of a
// cycle (x = b - D x) and the next cycle's start
__global__ __launch_bounds__(256) void k_cycle(KrylovDims dm, const double2* __restrict__ part,
                                               RhsState* __restrict__ st, int mode, CycleArgs ca) {
  const int r = blockIdx.x;
  if (!st[r].active) return;
  __shared__ double2 nr[KMAXV], scratch[8 * KMAXV];
  sum_blocks(part + int64_t(r) * dm.nblk * KMAXV, dm.nblk, 1, nr, scratch);
  if (threadIdx.x != 0) return;
  const double nrm = sqrt(nr[0].x);
  if (mode == 1) {
    RhsState s = {};
    s.bnorm = nrm;
    s.true_res = 1.0;
    if (!finite_d(nrm)) { s.nonfinite = 1; s.done = 1; }
    else if (nrm == 0.0) { s.converged = 1; s.done = 1; s.true_res = 0.0; }
    s.active = s.done ? 0 : 1;
    s.in_cycle = s.active;
    st[r] = s;
  } else {
    RhsState s = st[r];
    begin_cycle(dm, s, r, nrm, mode == 2, ca);
    st[r] = s;
  }
}

__global__ __launch_bounds__(256) void k_scale_next(KrylovDims dm, const double2* __restrict__ w,
                                                    double2* __restrict__ v,
                                                    const RhsState* __restrict__ st) {
  const int r = blockIdx.y;
  if (!st[r].active) return;
  const double inv = st[r].inv_h;
  const int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (d < dm.n) v[r * dm.n + d] = cscale(w[r * dm.n + d], inv);
}

// y = R^{-1} g (k x k upper triangle of the rotated Hessenberg matrix); marks the rhs for the
// x update and the true residual (active = in_cycle).
__global__ void k_backsolve(KrylovDims dm, RhsState* __restrict__ st, const double2* __restrict__ H,
                            const double2* __restrict__ g, double2* __restrict__ y) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= dm.nrhs) return;
  RhsState s = st[r];
  const int m = dm.m;
  if (!s.in_cycle || s.k == 0 || s.nonfinite) { s.active = s.in_cycle && !s.nonfinite; st[r] = s; return; }
  const double2* Hr = H + int64_t(r) * (m + 1) * m;
  const double2* gr = g + int64_t(r) * (m + 1);
  double2* yr = y + int64_t(r) * m;
  for (int i = s.k - 1; i >= 0; --i) {
    double2 acc = gr[i];
    for (int q = i + 1; q < s.k; ++q) acc = csub(acc, cmul(Hr[i * m + q], yr[q]));
    const double2 d = Hr[i * m + i];
    const double den = cabs2(d);
    yr[i] = cmul(acc, make_double2(d.x / den, -d.y / den));
  }
  s.active = 1;
  st[r] = s;
}

// x += sum_{i<k} Z_i y_i
template <typename Vz>
__global__ __launch_bounds__(256) void k_update_x(KrylovDims dm, const RhsState* __restrict__ st,
                                                  const double2* __restrict__ y,
                                                  const Vz* __restrict__ Z, int64_t zsj,
                                                  double2* __restrict__ x) {
  const int r = blockIdx.y;
  const RhsState& s = st[r];
  if (!s.active || s.k == 0) return;
  const int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (d >= dm.n) return;
  double2 acc = x[r * dm.n + d];
  const double2* yr = y + int64_t(r) * dm.m;
  for (int i = 0; i < s.k; ++i) acc = cfma(cconv<double2>(Z[i * zsj + r * dm.n + d]), yr[i], acc);
  x[r * dm.n + d] = acc;
}

// ------------------------------------------------------------------------------ launchers

using KFn = void (*)(hipStream_t, const KrylovDims&, const double2*, int64_t, double2*,
                    const double2*, double2*, const RhsState*);

template <int NV> void launch_dots(hipStream_t s, const KrylovDims& d, const double2* V, int64_t vsj,
                                   double2* w, const double2*, double2* part, const RhsState* st) {
  AMAMG_LAUNCH((k_dots<NV>), dim3(d.nblk, d.nrhs), dim3(256), 0, s, d, V, vsj, w, part, st);
}
template <int NV>
void launch_update_norm(hipStream_t s, const KrylovDims& d, const double2* V, int64_t vsj, double2* w,
                        const double2* hpart, double2* part, const RhsState* st) {
  AMAMG_LAUNCH((k_update_norm<NV>), dim3(d.nblk, d.nrhs), dim3(256), 0, s, d, V, vsj, w, hpart,
                     part, st);
}
template <int NV>
void launch_update_dots(hipStream_t s, const KrylovDims& d, const double2* V, int64_t vsj, double2* w,
                        const double2* hpart, double2* part, const RhsState* st) {
  AMAMG_LAUNCH((k_update_dots<NV, update_lanes(NV)>), dim3(d.nblk, d.nrhs), dim3(256), 0, s, d,
                     V, vsj, w, hpart, part, st);
}
template <int... I>
static constexpr std::array<KFn, sizeof...(I)> table_dots(std::integer_sequence<int, I...>) {
  return {&launch_dots<I + 1>...};
}
template <int... I>
static constexpr std::array<KFn, sizeof...(I)> table_update_dots(std::integer_sequence<int, I...>) {
  return {&launch_update_dots<I + 1>...};
}
template <int... I>
static constexpr std::array<KFn, sizeof...(I)> table_update_norm(std::integer_sequence<int, I...>) {
  return {&launch_update_norm<I + 1>...};
}
static const auto kDots = table_dots(std::make_integer_sequence<int, KMAXV>{});
static const auto kUpdDots = table_update_dots(std::make_integer_sequence<int, KMAXV>{});
static const auto kUpdNorm = table_update_norm(std::make_integer_sequence<int, KMAXV>{});

void dots(hipStream_t s, const KrylovDims& d, const double2* V, int64_t vsj, int nv,
          const double2* w, double2* part, const RhsState* st) {
  kDots[nv - 1](s, d, V, vsj, const_cast<double2*>(w), nullptr, part, st);
}

void update_dots(hipStream_t s, const KrylovDims& d, const double2* V, int64_t vsj, int nv,
                 double2* w, const double2* hpart, double2* part, const RhsState* st) {
  kUpdDots[nv - 1](s, d, V, vsj, w, hpart, part, st);
}

void update_norm(hipStream_t s, const KrylovDims& d, const double2* V, int64_t vsj, int nv,
                 double2* w, const double2* hpart, double2* part, const RhsState* st) {
  kUpdNorm[nv - 1](s, d, V, vsj, w, hpart, part, st);
}

void arnoldi(hipStream_t s, const KrylovDims& d, const double2* p1, const double2* p2,
             const double2* p3, RhsState* st, double2* H, double* cs, double2* sn, double2* g,
             int j, double tol, double inner_tol, int max_iters, double2* hist, int hist_cap) {
  ArnoldiArgs aa{H, cs, sn, g, j, tol, inner_tol, max_iters, hist, hist_cap};
  hipLaunchKernelGGL(k_arnoldi, dim3(d.nrhs), dim3(256), 0, s, d, p1, p2, p3, st, aa, j + 1);
}

void norm_control(hipStream_t s, const KrylovDims& d, const double2* x, double2* part, RhsState* st,
                  int mode, double2* g, double tol, int max_iters, double2* hist, int hist_cap) {
  CycleArgs ca{g, tol, max_iters, hist, hist_cap};
  hipLaunchKernelGGL(k_norm, dim3(d.nblk, d.nrhs), dim3(256), 0, s, d, x, part, st);
  hipLaunchKernelGGL(k_cycle, dim3(d.nrhs), dim3(256), 0, s, d, part, st, mode, ca);
}

__global__ void k_merge_states(RhsState* __restrict__ st, const RhsState* __restrict__ st2,
                               const int* __restrict__ admit, int cap) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < cap && admit[r]) st[r] = st2[r];
}

void merge_states(hipStream_t s, RhsState* st, const RhsState* st2, const int* admit, int cap) {
  hipLaunchKernelGGL(k_merge_states, dim3((cap + 63) / 64), dim3(64), 0, s, st, st2, admit, cap);
}

void scale_next(hipStream_t s, const KrylovDims& d, const double2* w, double2* v, const RhsState* st) {
  hipLaunchKernelGGL(k_scale_next, dim3(unsigned((d.n + 255) / 256), d.nrhs), dim3(256), 0, s, d, w, v, st);
}

void backsolve_update(hipStream_t s, const KrylovDims& d, RhsState* st, const double2* H,
                      const double2* g, double2* y, Real zprec, const void* Z, int64_t zsj,
                      double2* x) {
  hipLaunchKernelGGL(k_backsolve, dim3((d.nrhs + 63) / 64), dim3(64), 0, s, d, st, H, g, y);
  dim3 grid(unsigned((d.n + 255) / 256), d.nrhs);
  if (zprec == F64)
    hipLaunchKernelGGL((k_update_x<double2>), grid, dim3(256), 0, s, d, st, y, (const double2*)Z, zsj, x);
  else
    hipLaunchKernelGGL((k_update_x<float2>), grid, dim3(256), 0, s, d, st, y, (const float2*)Z, zsj, x);
}

}  // namespace amamg
