// Coarse-level kernels: block-stencil apply (Galerkin operator P^H A P, paper's Multilevel
// approach section), its 16-colour point-block Gauss-Seidel sweep, and the dense coarsest solve.
//
// A coarse operator is stored as a 5 x 5 block stencil: node n couples to n + (dt, dx),
// dt, dx in [-2, 2], through a b x b complex block A[n][(dt+2)*5 + (dx+2)][i][j] (node-major:
// everything a node needs is contiguous).  Coarse vectors are [rhs][node][b] complex.
#include "launch.hpp"

namespace amamg {

__device__ inline int wrapi(int v, int L) { v %= L; return v < 0 ? v + L : v; }

// One thread per (node, row i): y[n][i] = sum_d sum_j A[n][d][i][j] x[n+d][j]  (or f - that)
template <typename R, typename M, typename Vin, typename Vout>
__global__ __launch_bounds__(256) void k_stencil_apply(const M* __restrict__ A,
                                                       const Vin* __restrict__ x,
                                                       Vout* __restrict__ y,
                                                       const Vout* __restrict__ f, int Lt, int Lx,
                                                       int b, int64_t stride,
                                                       const RhsState* __restrict__ st) {
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  const int64_t gid = int64_t(xcd_block(blockIdx.x, gridDim.x)) * 256 + threadIdx.x;
  if (gid >= int64_t(Lt) * Lx * b) return;
  using C = cplx<R>;
  const int n = int(gid / b), i = int(gid - int64_t(n) * b);
  const int t = n / Lx, xc = n - t * Lx;
  const Vin* xr = x + r * stride;
  const M* An = A + int64_t(n) * 25 * b * b + int64_t(i) * b;
  C acc = czero<R>();
  for (int dt = -2; dt <= 2; ++dt) {
    const int tt = wrapi(t + dt, Lt);
    for (int dx = -2; dx <= 2; ++dx) {
      const int m = tt * Lx + wrapi(xc + dx, Lx);
      const M* blk = An + int64_t((dt + 2) * 5 + (dx + 2)) * b * b;
      const Vin* xm = xr + int64_t(m) * b;
      for (int j = 0; j < b; ++j) acc = cfma(cconv<C>(blk[j]), cconv<C>(xm[j]), acc);
    }
  }
  Vout* yr = y + r * stride;
  if (f) acc = csub(cconv<C>(f[r * stride + gid]), acc);
  yr[gid] = cconv<Vout>(acc);
}

// Colour c = (I mod 4) * 4 + (J mod 4); nodes of one colour do not couple (stencil reach 2).
// Lanes of one node sit in one wavefront (b divides 64), so the b-vector of residuals is
// exchanged with shuffles before applying Dinv_n.
template <typename R, typename M, typename Vx>
__global__ __launch_bounds__(256) void k_stencil_gs(const M* __restrict__ A,
                                                    const M* __restrict__ Dinv, Vx* x,
                                                    const Vx* __restrict__ f, int Lt, int Lx,
                                                    int b, int colour, int64_t stride,
                                                    const RhsState* __restrict__ st) {
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  const int gid = blockIdx.x * 256 + threadIdx.x;
  const int qx = Lx >> 2;
  const int ncn = (Lt >> 2) * qx;                 // nodes of this colour
  const int k = gid / b, i = gid - (gid / b) * b;
  const bool live = k < ncn;
  using C = cplx<R>;
  C res = czero<R>();
  int n = 0;
  if (live) {
    const int ct = colour >> 2, cx = colour & 3;
    const int t = 4 * (k / qx) + ct, xc = 4 * (k % qx) + cx;
    n = t * Lx + xc;
    const Vx* xr = x + r * stride;
    const M* An = A + int64_t(n) * 25 * b * b + int64_t(i) * b;
    if (f) res = cconv<C>(f[r * stride + int64_t(n) * b + i]);
    for (int dt = -2; dt <= 2; ++dt) {
      const int tt = wrapi(t + dt, Lt);
      for (int dx = -2; dx <= 2; ++dx) {
        if (dt == 0 && dx == 0) continue;
        const int m = tt * Lx + wrapi(xc + dx, Lx);
        const M* blk = An + int64_t((dt + 2) * 5 + (dx + 2)) * b * b;
        const Vx* xm = xr + int64_t(m) * b;
        for (int j = 0; j < b; ++j) res = csub(res, cmul(cconv<C>(blk[j]), cconv<C>(xm[j])));
      }
    }
  }
  // x_n[i] = sum_j Dinv[n][i][j] res_j, res_j held by lane (lane - i + j)
  const int lane = threadIdx.x & (AMAMG_WAVE - 1);
  const int base = lane - i;
  C out = czero<R>();
  const M* Dn = Dinv + int64_t(n) * b * b + int64_t(i) * b;
  for (int j = 0; j < b; ++j) {
    R re = __shfl(res.x, base + j), im = __shfl(res.y, base + j);
    if (live) out = cfma(cconv<C>(Dn[j]), mk<R>(re, im), out);
  }
  if (live) x[r * stride + int64_t(n) * b + i] = cconv<Vx>(out);
}

// y = Ainv v for the coarsest level (matrix FP64): 64 lanes per row, 4 rows per block.
template <typename Vin, typename Vout>
__global__ __launch_bounds__(256) void k_dense_apply(const double2* __restrict__ Ainv,
                                                     const Vin* __restrict__ v,
                                                     Vout* __restrict__ y, int n,
                                                     int64_t stride,
                                                     const RhsState* __restrict__ st) {
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  double re = 0, im = 0;
  if (row < n) {
    const double2* Ar = Ainv + int64_t(row) * n;
    const Vin* vr = v + r * stride;
    double2 acc = make_double2(0, 0);
    for (int j = lane; j < n; j += 64) acc = cfma(Ar[j], cconv<double2>(vr[j]), acc);
    re = acc.x; im = acc.y;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (row < n && lane == 0) y[r * stride + row] = cconv<Vout>(make_double2(re, im));
}

// ------------------------------------------------------------------------------ launchers

void stencil_apply(hipStream_t s, Real prec, const void* A, const void* x, void* y, const void* f,
                   int Lt, int Lx, int b, int nrhs, int64_t stride, const RhsState* st) {
  dim3 g(unsigned((int64_t(Lt) * Lx * b + 255) / 256), unsigned(nrhs));
  if (prec == F64)
    hipLaunchKernelGGL((k_stencil_apply<double, double2, double2, double2>), g, dim3(256), 0, s,
                       (const double2*)A, (const double2*)x, (double2*)y, (const double2*)f, Lt,
                       Lx, b, stride, st);
  else
    hipLaunchKernelGGL((k_stencil_apply<float, float2, float2, float2>), g, dim3(256), 0, s,
                       (const float2*)A, (const float2*)x, (float2*)y, (const float2*)f, Lt, Lx,
                       b, stride, st);
}

void stencil_gs(hipStream_t s, Real prec, const void* A, const void* Dinv, void* x, const void* f,
                int Lt, int Lx, int b, int colour, int nrhs, int64_t stride, const RhsState* st) {
  const int ncn = (Lt / 4) * (Lx / 4);
  dim3 g(unsigned((ncn * b + 255) / 256), unsigned(nrhs));
  if (prec == F64)
    hipLaunchKernelGGL((k_stencil_gs<double, double2, double2>), g, dim3(256), 0, s,
                       (const double2*)A, (const double2*)Dinv, (double2*)x, (const double2*)f, Lt,
                       Lx, b, colour, stride, st);
  else
    hipLaunchKernelGGL((k_stencil_gs<float, float2, float2>), g, dim3(256), 0, s,
                       (const float2*)A, (const float2*)Dinv, (float2*)x, (const float2*)f, Lt, Lx,
                       b, colour, stride, st);
}

void dense_apply(hipStream_t s, Real prec, const double2* Ainv, const void* v, void* y, int n,
                 int nrhs, int64_t stride, const RhsState* st) {
  dim3 g(unsigned((n + 3) / 4), unsigned(nrhs));
  if (prec == F64)
    hipLaunchKernelGGL((k_dense_apply<double2, double2>), g, dim3(256), 0, s, Ainv,
                       (const double2*)v, (double2*)y, n, stride, st);
  else
    hipLaunchKernelGGL((k_dense_apply<float2, float2>), g, dim3(256), 0, s, Ainv,
                       (const float2*)v, (float2*)y, n, stride, st);
}

}  // namespace amamg
