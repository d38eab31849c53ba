// FGMRES(m) kernels, FP64 (paper: FGMRES outer solver, relative tolerance 1e-10).
//
// Right-preconditioned flexible Arnoldi with classical Gram-Schmidt applied twice.  All
// reductions are two-pass and fixed-order (per-block partial sums, then a sum over blocks in
// block order), so results are bitwise reproducible.  Givens rotation for (a, b) =
// (H_jj, H_{j+1,j}): nu = sqrt(|a|^2 + |b|^2), c = |a| / nu, s = (a / |a|) conj(b) / nu
// (c = 0, s = 1 when a = 0); a rotation maps (x, y) -> (c x + s y, -conj(s) x + c y).
//
// Vector layouts: basis V [j][rhs][n], search directions Z [j][rhs][n], w and x [rhs][n].
// Scalars per right-hand side live in RhsState and small arrays on the device; the host
// reads them once per cycle.
#include "launch.hpp"

namespace amamg {

#define KMAXV 32

template <int NV>
__device__ inline void block_reduce_store(double2 (&acc)[NV], int nv, double2* out, double* lds) {
  // lds: 2 * NV * 4 doubles
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if (i < nv) {
      double re = wave_sum(acc[i].x), im = wave_sum(acc[i].y);
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

// part[r][blk][i] = sum_{d in block} conj(V_i[r][d]) w[r][d]
__global__ __launch_bounds__(256) void k_dots_partial(KrylovDims dm, const double2* __restrict__ V,
                                                      int64_t vsj, int nv,
                                                      const double2* __restrict__ w,
                                                      double2* __restrict__ part,
                                                      const RhsState* __restrict__ st) {
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  __shared__ double lds[2 * KMAXV * 4];
  double2 acc[KMAXV];
#pragma unroll
  for (int i = 0; i < KMAXV; ++i) acc[i] = make_double2(0, 0);
  const double2* wr = w + r * dm.n;
  const double2* Vr = V + r * dm.n;
  for (int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x; d < dm.n; d += int64_t(gridDim.x) * 256) {
    const double2 wd = wr[d];
#pragma unroll
    for (int i = 0; i < KMAXV; ++i)
      if (i < nv) acc[i] = cfmac(Vr[i * vsj + d], wd, acc[i]);
  }
  block_reduce_store<KMAXV>(acc, nv, part + (int64_t(r) * gridDim.x + blockIdx.x) * KMAXV, lds);
}

// w -= sum_i V_i h_i, then (mode 1) part = V^H w_new, or (mode 2) part[0] = |w_new|^2
__global__ __launch_bounds__(256) void k_update_partial(KrylovDims dm, const double2* __restrict__ V,
                                                        int64_t vsj, int nv, double2* __restrict__ w,
                                                        const double2* __restrict__ h, int hstride,
                                                        double2* __restrict__ part, int mode,
                                                        const RhsState* __restrict__ st) {
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  __shared__ double lds[2 * KMAXV * 4];
  __shared__ double2 hs[KMAXV];
  if (threadIdx.x < nv) hs[threadIdx.x] = h[r * hstride + threadIdx.x];
  __syncthreads();
  double2 acc[KMAXV];
#pragma unroll
  for (int i = 0; i < KMAXV; ++i) acc[i] = make_double2(0, 0);
  double2* wr = w + r * dm.n;
  const double2* Vr = V + r * dm.n;
  for (int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x; d < dm.n; d += int64_t(gridDim.x) * 256) {
    double2 v[KMAXV];
    double2 wd = wr[d];
#pragma unroll
    for (int i = 0; i < KMAXV; ++i)
      if (i < nv) { v[i] = Vr[i * vsj + d]; wd = csub(wd, cmul(v[i], hs[i])); }
    wr[d] = wd;
    if (mode == 1) {
#pragma unroll
      for (int i = 0; i < KMAXV; ++i)
        if (i < nv) acc[i] = cfmac(v[i], wd, acc[i]);
    } else {
      acc[0].x += cabs2(wd);
    }
  }
  block_reduce_store<KMAXV>(acc, mode == 1 ? nv : 1, part + (int64_t(r) * gridDim.x + blockIdx.x) * KMAXV, lds);
}

// out[r*ostride + i] = sum over blocks (in block order) of part[r][blk][i]
__global__ void k_sum_partials(int nblk, const double2* __restrict__ part, int nv,
                               double2* __restrict__ out, int ostride,
                               const RhsState* __restrict__ st) {
  const int r = blockIdx.x;
  if (st && !st[r].active) return;
  const int i = threadIdx.x;
  if (i >= nv) return;
  double2 acc = make_double2(0, 0);
  for (int b = 0; b < nblk; ++b) acc = cadd(acc, part[(int64_t(r) * nblk + b) * KMAXV + i]);
  out[r * ostride + i] = acc;
}

__global__ __launch_bounds__(256) void k_norm_partial(KrylovDims dm, const double2* __restrict__ x,
                                                      double2* __restrict__ part,
                                                      const RhsState* __restrict__ st,
                                                      int only_active) {
  const int r = blockIdx.y;
  if (only_active && st && !st[r].active) return;
  __shared__ double lds[2 * KMAXV * 4];
  double2 acc[1] = {make_double2(0, 0)};
  const double2* xr = x + r * dm.n;
  for (int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x; d < dm.n; d += int64_t(gridDim.x) * 256)
    acc[0].x += cabs2(xr[d]);
  block_reduce_store<1>(acc, 1, part + (int64_t(r) * gridDim.x + blockIdx.x) * KMAXV, lds);
}

__device__ inline double part_norm(const double2* part, int r, int nblk) {
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t(r) * nblk + b) * KMAXV].x;
  return sqrt(s);
}

__device__ inline bool finite_d(double v) { return v == v && v - v == 0.0; }

// ||b|| and a fresh state per right-hand side
__global__ void k_init_states(KrylovDims dm, RhsState* __restrict__ st, const double2* __restrict__ part) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= dm.nrhs) return;
  RhsState s = {};
  s.bnorm = part_norm(part, r, dm.nblk);
  s.true_res = 1.0;
  if (!finite_d(s.bnorm)) { s.nonfinite = 1; s.done = 1; }
  else if (s.bnorm == 0.0) { s.converged = 1; s.done = 1; s.true_res = 0.0; }
  s.active = s.done ? 0 : 1;   // the first residual is computed for every live rhs
  s.in_cycle = s.active;
  st[r] = s;
}

// Called with part = |r|^2 partials of r = b - D x (stored in V_0).  first: the residual of the
// start vector; otherwise the true residual after a cycle.  Starts the next cycle when needed.
__global__ void k_cycle_begin(KrylovDims dm, RhsState* __restrict__ st, const double2* __restrict__ part,
                              double2* __restrict__ g, double tol, int first, int max_iters,
                              double2* __restrict__ hist, int hist_cap) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= dm.nrhs) return;
  RhsState s = st[r];
  if (s.done || !s.in_cycle || s.nonfinite) {
    if (s.nonfinite) s.done = 1;
    s.active = 0; s.in_cycle = 0; st[r] = s; return;
  }
  const double beta = part_norm(part, r, dm.nblk);
  s.true_res = beta / s.bnorm;
  if (!finite_d(beta)) { s.nonfinite = 1; s.done = 1; s.active = 0; s.in_cycle = 0; st[r] = s; return; }
  if (!first && s.hist_len < hist_cap) hist[int64_t(r) * hist_cap + s.hist_len++] = make_double2(s.true_res, 1.0);
  if (beta <= tol * s.bnorm) {
    s.converged = 1; s.done = 1; s.active = 0; s.in_cycle = 0;
  } else if (s.iters >= max_iters) {
    s.done = 1; s.active = 0; s.in_cycle = 0;
  } else {
    if (!first) s.restarts += 1;
    s.beta = beta;
    s.inv_h = 1.0 / beta;
    s.k = 0;
    s.active = 1;
    s.in_cycle = 1;
    double2* gr = g + int64_t(r) * (dm.m + 1);
    gr[0] = make_double2(beta, 0.0);
    for (int i = 1; i <= dm.m; ++i) gr[i] = make_double2(0, 0);
  }
  st[r] = s;
}

// Arnoldi step j: new Hessenberg column, rotations, residual estimate, end-of-cycle test.
__global__ void k_arnoldi_finish(KrylovDims dm, RhsState* __restrict__ st, const double2* __restrict__ part,
                                 const double2* __restrict__ h1, const double2* __restrict__ h2,
                                 double2* __restrict__ H, double* __restrict__ cs,
                                 double2* __restrict__ sn, double2* __restrict__ g, int j,
                                 double tol, double inner_tol, int max_iters,
                                 double2* __restrict__ hist, int hist_cap) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= dm.nrhs) return;
  RhsState s = st[r];
  if (!s.active) return;
  const int m = dm.m;
  double2* Hr = H + int64_t(r) * (m + 1) * m;     // H[i][j] at i*m + j
  double* csr = cs + int64_t(r) * m;
  double2* snr = sn + int64_t(r) * m;
  double2* gr = g + int64_t(r) * (m + 1);
  const double hn = part_norm(part, r, dm.nblk);
  for (int i = 0; i <= j; ++i) Hr[i * m + j] = cadd(h1[r * KMAXV + i], h2[r * KMAXV + i]);
  Hr[(j + 1) * m + j] = make_double2(hn, 0.0);
  for (int i = 0; i < j; ++i) {
    const double2 x = Hr[i * m + j], y = Hr[(i + 1) * m + j];
    const double c = csr[i];
    const double2 sv = snr[i];
    Hr[i * m + j] = cadd(cscale(x, c), cmul(sv, y));
    Hr[(i + 1) * m + j] = csub(cscale(y, c), cmulc(sv, x));
  }
  const double2 a = Hr[j * m + j], bb = Hr[(j + 1) * m + j];
  double c;
  double2 sv;
  const double aa = sqrt(cabs2(a));
  if (aa == 0.0) {
    c = 0.0;
    sv = make_double2(1.0, 0.0);
  } else {
    const double nu = sqrt(cabs2(a) + cabs2(bb));
    c = aa / nu;
    sv = cscale(cmul(make_double2(a.x / aa, a.y / aa), cconj(bb)), 1.0 / nu);
  }
  Hr[j * m + j] = cadd(cscale(a, c), cmul(sv, bb));
  Hr[(j + 1) * m + j] = make_double2(0, 0);
  csr[j] = c;
  snr[j] = sv;
  const double2 gj = gr[j];
  gr[j + 1] = cscale(cmulc(sv, gj), -1.0);
  gr[j] = cscale(gj, c);
  s.iters += 1;
  s.k = j + 1;
  const double gabs = sqrt(cabs2(gr[j + 1]));
  s.est = gabs / s.bnorm;
  if (s.hist_len < hist_cap) hist[int64_t(r) * hist_cap + s.hist_len++] = make_double2(s.est, 0.0);
  bool end = (gabs <= tol * s.bnorm) || (hn <= 1e-300 * s.bnorm) || (s.iters >= max_iters) ||
             (j + 1 == m) || (inner_tol > 0.0 && gabs <= inner_tol * s.beta);
  if (!finite_d(hn) || !finite_d(gabs)) { s.nonfinite = 1; end = true; }
  if (end) s.active = 0;
  else s.inv_h = 1.0 / hn;
  st[r] = s;
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

__global__ void k_copy(const double2* __restrict__ x, double2* __restrict__ y, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

// ------------------------------------------------------------------------------ launchers

void dots_partial(hipStream_t s, const KrylovDims& d, const double2* V, int64_t vsj, int nv,
                  const double2* w, double2* part, const RhsState* st) {
  hipLaunchKernelGGL(k_dots_partial, dim3(d.nblk, d.nrhs), dim3(256), 0, s, d, V, vsj, nv, w, part, st);
}

void update_partial(hipStream_t s, const KrylovDims& d, const double2* V, int64_t vsj, int nv,
                    double2* w, const double2* h, int hstride, double2* part, int mode,
                    const RhsState* st) {
  hipLaunchKernelGGL(k_update_partial, dim3(d.nblk, d.nrhs), dim3(256), 0, s, d, V, vsj, nv, w, h,
                     hstride, part, mode, st);
}

void sum_partials(hipStream_t s, const KrylovDims& d, const double2* part, int nv, double2* out,
                  int ostride, const RhsState* st) {
  hipLaunchKernelGGL(k_sum_partials, dim3(d.nrhs), dim3(64), 0, s, d.nblk, part, nv, out, ostride, st);
}

void norm_partial(hipStream_t s, const KrylovDims& d, const double2* x, double2* part,
                  const RhsState* st, int only_active) {
  hipLaunchKernelGGL(k_norm_partial, dim3(d.nblk, d.nrhs), dim3(256), 0, s, d, x, part, st, only_active);
}

void init_states(hipStream_t s, const KrylovDims& d, RhsState* st, const double2* part) {
  hipLaunchKernelGGL(k_init_states, dim3((d.nrhs + 63) / 64), dim3(64), 0, s, d, st, part);
}

void cycle_begin(hipStream_t s, const KrylovDims& d, RhsState* st, const double2* part, double2* g,
                 double tol, int first, int max_iters, double2* hist, int hist_cap) {
  hipLaunchKernelGGL(k_cycle_begin, dim3((d.nrhs + 63) / 64), dim3(64), 0, s, d, st, part, g, tol,
                     first, max_iters, hist, hist_cap);
}

void arnoldi_finish(hipStream_t s, const KrylovDims& d, RhsState* st, const double2* part,
                    const double2* h1, const double2* h2, double2* H, double* cs, double2* sn,
                    double2* g, int j, double tol, double inner_tol, int max_iters,
                    double2* hist, int hist_cap) {
  hipLaunchKernelGGL(k_arnoldi_finish, dim3((d.nrhs + 63) / 64), dim3(64), 0, s, d, st, part, h1, h2,
                     H, cs, sn, g, j, tol, inner_tol, max_iters, hist, hist_cap);
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

void copy_vec(hipStream_t s, const double2* x, double2* y, int64_t n) {
  hipLaunchKernelGGL(k_copy, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, x, y, n);
}

void zero_vec(hipStream_t s, void* x, int64_t bytes) { (void)hipMemsetAsync(x, 0, bytes, s); }

}  // namespace amamg
