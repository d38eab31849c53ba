// Fine-level kernels: the Wilson-Dirac stencil of the Schwinger model (paper, Schwinger Model
// subsection) and its red-black point Gauss-Seidel sweep.
//
// (D psi)(n) = (m0 + 2) psi(n) - 1/2 sum_mu [ (1 - sigma_mu) U_mu(n) psi(n + mu)
//                                            + (1 + sigma_mu) U_mu(n - mu)^* psi(n - mu) ]
// sigma_0 = [[0,1],[1,0]], sigma_1 = [[0,-i],[i,0]]; mu = 0 is time; the fermion picks up a
// factor -1 on hops across the time boundary (antiperiodic), space is periodic.
// The spin projectors have rank one:
//   (1 - sigma_0) psi = (psi0 - psi1) (1, -1)     (1 + sigma_0) psi = (psi0 + psi1) (1, 1)
//   (1 - sigma_1) psi = (psi0 + i psi1) (1, -i)   (1 + sigma_1) psi = (psi0 - i psi1) (1, i)
// so each hop costs one complex projection, one link multiply and two accumulations.
//
// Layout: one thread per site, site = t * nx + x; a field is [rhs][site][2 spin] complex.
// Bytes per site (FP64): 4 neighbour spinors + own (cache-reused: 32 B from HBM), 2 links
// (32 B), result (32 B) = 96 B; about 60 flops.
#include "launch.hpp"

namespace amamg {

template <typename R, typename L, typename Vin>
__device__ inline void wilson_hops(const L* __restrict__ U0, const L* __restrict__ U1,
                                   const Vin* __restrict__ x, int t, int xc, int nt, int nx,
                                   cplx<R>& o0, cplx<R>& o1) {
  using C = cplx<R>;
  const int n = t * nx + xc;
  const int tf = (t + 1 == nt) ? 0 : t + 1, tb = (t == 0) ? nt - 1 : t - 1;
  const int xf = (xc + 1 == nx) ? 0 : xc + 1, xb = (xc == 0) ? nx - 1 : xc - 1;
  const int nf0 = tf * nx + xc, nb0 = tb * nx + xc, nf1 = t * nx + xf, nb1 = t * nx + xb;
  const R sf = (t == nt - 1) ? R(-1) : R(1);
  const R sb = (t == 0) ? R(-1) : R(1);
  // forward time hop
  C a0 = cconv<C>(x[2 * nf0]), a1 = cconv<C>(x[2 * nf0 + 1]);
  C h = cscale(cmul(load_link<R>(U0, n), csub(a0, a1)), sf);
  C s0 = h, s1 = mk<R>(-h.x, -h.y);
  // backward time hop
  C b0 = cconv<C>(x[2 * nb0]), b1 = cconv<C>(x[2 * nb0 + 1]);
  h = cscale(cmulc(load_link<R>(U0, nb0), cadd(b0, b1)), sb);
  s0 = cadd(s0, h);
  s1 = cadd(s1, h);
  // forward space hop: (1, -i) (psi0 + i psi1)
  C c0 = cconv<C>(x[2 * nf1]), c1 = cconv<C>(x[2 * nf1 + 1]);
  h = cmul(load_link<R>(U1, n), cadd(c0, ctimes_i(c1)));
  s0 = cadd(s0, h);
  s1 = csub(s1, ctimes_i(h));
  // backward space hop: (1, i) (psi0 - i psi1)
  C d0 = cconv<C>(x[2 * nb1]), d1 = cconv<C>(x[2 * nb1 + 1]);
  h = cmulc(load_link<R>(U1, nb1), csub(d0, ctimes_i(d1)));
  s0 = cadd(s0, h);
  s1 = cadd(s1, ctimes_i(h));
  o0 = cscale(s0, R(-0.5));
  o1 = cscale(s1, R(-0.5));
}

template <typename R, typename L, typename Vin, typename Vout>
__global__ __launch_bounds__(256) void k_wilson_apply(const L* __restrict__ U0,
                                                      const L* __restrict__ U1,
                                                      const Vin* __restrict__ x,
                                                      Vout* __restrict__ y,
                                                      const double2* __restrict__ b, int nt,
                                                      int nx, R mp2, int64_t stride,
                                                      const RhsState* __restrict__ st) {
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  const int n = xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (n >= nt * nx) return;
  using C = cplx<R>;
  const Vin* xr = x + r * stride;
  const int t = n / nx, xc = n - t * nx;
  C o0, o1;
  wilson_hops<R, L, Vin>(U0, U1, xr, t, xc, nt, nx, o0, o1);
  C p0 = cconv<C>(xr[2 * n]), p1 = cconv<C>(xr[2 * n + 1]);
  C y0 = cadd(cscale(p0, mp2), o0), y1 = cadd(cscale(p1, mp2), o1);
  Vout* yr = y + r * stride;
  if (b) {
    const double2* br = b + r * stride;
    // residual in FP64
    double2 e0 = cconv<double2>(y0), e1 = cconv<double2>(y1);
    yr[2 * n] = cconv<Vout>(csub(br[2 * n], e0));
    yr[2 * n + 1] = cconv<Vout>(csub(br[2 * n + 1], e1));
  } else {
    yr[2 * n] = cconv<Vout>(y0);
    yr[2 * n + 1] = cconv<Vout>(y1);
  }
}

// Sites of one colour c = (t + x) mod 2: x(n) <- x(n) + (b(n) - (D x)(n)) / (m0 + 2), which
// equals (b(n) - hops(n)) / (m0 + 2) because the diagonal of D at n is (m0 + 2) I.
template <typename R, typename L, typename Vx>
__global__ __launch_bounds__(256) void k_wilson_gs(const L* __restrict__ U0,
                                                   const L* __restrict__ U1, Vx* x,
                                                   const double2* __restrict__ b, int nt,
                                                   int nx, R inv_mp2, int colour, int64_t stride,
                                                   const RhsState* __restrict__ st) {
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  const int idx = xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  const int half = nx >> 1;
  if (idx >= nt * half) return;
  using C = cplx<R>;
  const int t = idx / half;
  const int xc = 2 * (idx - t * half) + ((t + colour) & 1);
  const int n = t * nx + xc;
  Vx* xr = x + r * stride;
  C o0, o1;
  wilson_hops<R, L, Vx>(U0, U1, xr, t, xc, nt, nx, o0, o1);
  C f0 = czero<R>(), f1 = czero<R>();
  if (b) {
    const double2* br = b + r * stride;
    f0 = cconv<C>(br[2 * n]);
    f1 = cconv<C>(br[2 * n + 1]);
  }
  xr[2 * n] = cconv<Vx>(cscale(csub(f0, o0), inv_mp2));
  xr[2 * n + 1] = cconv<Vx>(cscale(csub(f1, o1), inv_mp2));
}

__global__ void k_build_fine_stencil(const double2* __restrict__ U0, const double2* __restrict__ U1,
                                     int nt, int nx, double m0, double2* __restrict__ A) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nt * nx) return;
  const int t = n / nx, xc = n - t * nx;
  const int tb = (t == 0) ? nt - 1 : t - 1, xb = (xc == 0) ? nx - 1 : xc - 1;
  const double sf = (t == nt - 1) ? -1.0 : 1.0, sb = (t == 0) ? -1.0 : 1.0;
  double2* blk = A + int64_t(n) * 5 * 4;
  // offset 0: (m0 + 2) I
  blk[0] = make_double2(m0 + 2.0, 0.0); blk[1] = make_double2(0, 0);
  blk[2] = make_double2(0, 0);          blk[3] = make_double2(m0 + 2.0, 0.0);
  // offset (+1,0): -1/2 s U0(n) (1 - sigma0) = -1/2 s U0 [[1,-1],[-1,1]]
  double2 u = cscale(U0[n], -0.5 * sf);
  blk[4] = u; blk[5] = cscale(u, -1.0); blk[6] = cscale(u, -1.0); blk[7] = u;
  // offset (-1,0): -1/2 s conj(U0(n - t)) (1 + sigma0) = ... [[1,1],[1,1]]
  u = cscale(cconj(U0[tb * nx + xc]), -0.5 * sb);
  blk[8] = u; blk[9] = u; blk[10] = u; blk[11] = u;
  // offset (0,+1): -1/2 U1(n) (1 - sigma1) = -1/2 U1 [[1, i], [-i, 1]]
  u = cscale(U1[n], -0.5);
  blk[12] = u; blk[13] = ctimes_i(u); blk[14] = cscale(ctimes_i(u), -1.0); blk[15] = u;
  // offset (0,-1): -1/2 conj(U1(n - x)) (1 + sigma1) = ... [[1, -i], [i, 1]]
  u = cscale(cconj(U1[t * nx + xb]), -0.5);
  blk[16] = u; blk[17] = cscale(ctimes_i(u), -1.0); blk[18] = ctimes_i(u); blk[19] = u;
}

__global__ void k_links_f32(const double2* __restrict__ U, float2* __restrict__ out, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2(float(U[i].x), float(U[i].y));
}

__global__ void k_links_bf16(const double2* __restrict__ U, bf16c* __restrict__ out, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    uint32_t re = f32_to_bf16_rne(float(U[i].x)), im = f32_to_bf16_rne(float(U[i].y));
    out[i].bits = re | (im << 16);
  }
}

template <typename A, typename B>
__global__ void k_cast(const A* __restrict__ x, B* __restrict__ y, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = cconv<B>(x[i]);
}

// ------------------------------------------------------------------------------ launchers

static inline dim3 grid1(int64_t n, int nrhs) { return dim3(unsigned((n + 255) / 256), unsigned(nrhs)); }

template <typename R, typename L, typename Vin, typename Vout>
static void wilson_apply_t(hipStream_t s, const void* U0, const void* U1, const void* x, void* y,
                           const double2* b, int nt, int nx, double m0, int nrhs, int64_t stride,
                           const RhsState* st) {
  hipLaunchKernelGGL((k_wilson_apply<R, L, Vin, Vout>), grid1(int64_t(nt) * nx, nrhs), dim3(256), 0, s,
                     (const L*)U0, (const L*)U1, (const Vin*)x, (Vout*)y, b, nt, nx, R(m0 + 2.0),
                     stride, st);
}

void wilson_apply(hipStream_t s, LinkStore ls, const void* U0, const void* U1, Real vin,
                  const void* x, Real vout, void* y, const double2* b, int nt, int nx, double m0,
                  int nrhs, int64_t stride, const RhsState* st) {
  if (ls == LINK_F64) {
    if (vin == F64 && vout == F64) wilson_apply_t<double, double2, double2, double2>(s, U0, U1, x, y, b, nt, nx, m0, nrhs, stride, st);
    else if (vin == F32 && vout == F64) wilson_apply_t<double, double2, float2, double2>(s, U0, U1, x, y, b, nt, nx, m0, nrhs, stride, st);
    else wilson_apply_t<double, double2, double2, float2>(s, U0, U1, x, y, b, nt, nx, m0, nrhs, stride, st);
  } else if (ls == LINK_F32) {
    if (vin == F32 && vout == F64) wilson_apply_t<float, float2, float2, double2>(s, U0, U1, x, y, b, nt, nx, m0, nrhs, stride, st);
    else if (vin == F32 && vout == F32) wilson_apply_t<float, float2, float2, float2>(s, U0, U1, x, y, b, nt, nx, m0, nrhs, stride, st);
    else if (vin == F64 && vout == F64) wilson_apply_t<float, float2, double2, double2>(s, U0, U1, x, y, b, nt, nx, m0, nrhs, stride, st);
    else wilson_apply_t<float, float2, double2, float2>(s, U0, U1, x, y, b, nt, nx, m0, nrhs, stride, st);
  } else {
    if (vin == F32 && vout == F32) wilson_apply_t<float, bf16c, float2, float2>(s, U0, U1, x, y, b, nt, nx, m0, nrhs, stride, st);
    else wilson_apply_t<float, bf16c, float2, double2>(s, U0, U1, x, y, b, nt, nx, m0, nrhs, stride, st);
  }
}

template <typename R, typename L, typename Vx>
static void wilson_gs_t(hipStream_t s, const void* U0, const void* U1, void* x, const double2* b,
                        int nt, int nx, double m0, int colour, int nrhs, int64_t stride,
                        const RhsState* st) {
  hipLaunchKernelGGL((k_wilson_gs<R, L, Vx>), grid1(int64_t(nt) * (nx / 2), nrhs), dim3(256), 0, s,
                     (const L*)U0, (const L*)U1, (Vx*)x, b, nt, nx, R(1.0 / (m0 + 2.0)), colour,
                     stride, st);
}

void wilson_gs(hipStream_t s, LinkStore ls, const void* U0, const void* U1, Real vx, void* x,
               const double2* b, int nt, int nx, double m0, int colour, int nrhs, int64_t stride,
               const RhsState* st) {
  if (ls == LINK_F64 && vx == F64) wilson_gs_t<double, double2, double2>(s, U0, U1, x, b, nt, nx, m0, colour, nrhs, stride, st);
  else if (ls == LINK_F32) wilson_gs_t<float, float2, float2>(s, U0, U1, x, b, nt, nx, m0, colour, nrhs, stride, st);
  else wilson_gs_t<float, bf16c, float2>(s, U0, U1, x, b, nt, nx, m0, colour, nrhs, stride, st);
}

void build_fine_stencil(hipStream_t s, const double2* U0, const double2* U1, int nt, int nx,
                        double m0, double2* A0) {
  hipLaunchKernelGGL(k_build_fine_stencil, dim3((nt * nx + 255) / 256), dim3(256), 0, s, U0, U1, nt,
                     nx, m0, A0);
}

void links_to_f32(hipStream_t s, const double2* U, float2* out, int64_t n) {
  hipLaunchKernelGGL(k_links_f32, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, U, out, n);
}

void links_to_bf16(hipStream_t s, const double2* U, bf16c* out, int64_t n) {
  hipLaunchKernelGGL(k_links_bf16, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, U, out, n);
}

void cast_vec(hipStream_t s, Real from, const void* x, Real to, void* y, int64_t n) {
  dim3 g(unsigned((n + 255) / 256));
  if (from == F64 && to == F32) hipLaunchKernelGGL((k_cast<double2, float2>), g, dim3(256), 0, s, (const double2*)x, (float2*)y, n);
  else if (from == F32 && to == F64) hipLaunchKernelGGL((k_cast<float2, double2>), g, dim3(256), 0, s, (const float2*)x, (double2*)y, n);
  else if (from == F64) hipLaunchKernelGGL((k_cast<double2, double2>), g, dim3(256), 0, s, (const double2*)x, (double2*)y, n);
  else hipLaunchKernelGGL((k_cast<float2, float2>), g, dim3(256), 0, s, (const float2*)x, (float2*)y, n);
}

}  // namespace amamg
