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
// Layout: a field is [rhs][site][2 spin] complex, site = t * nx + x.  Each workgroup stages a
// tile of the field with its one-site halo in LDS (read from HBM once), then one thread per site
// applies the stencil.  Bytes per site (FP64): spinor 32 B, 2 links 32 B, result 32 B = 96 B;
// about 60 flops.
#include "launch.hpp"

namespace amamg {

// One site's two spin components, moved as one 16-byte (FP32) or two 16-byte (FP64) accesses;
// fields are 16-byte aligned.
template <typename V> struct alignas(16) Spinor { V s0, s1; };

template <typename To, typename From> __device__ inline Spinor<To> sconv(Spinor<From> a) {
  return Spinor<To>{cconv<To>(a.s0), cconv<To>(a.s1)};
}

// Spin-projected hops of one site, -1/2 sum_mu [(1 - sigma_mu) U_mu(n) psi(n + mu) +
// (1 + sigma_mu) U_mu(n - mu)^* psi(n - mu)], from its four neighbours; u0f = U0(n),
// u0b = U0(n - t), u1f = U1(n), u1b = U1(n - x); sf, sb are the time-boundary signs.
template <typename C, typename R>
__device__ inline Spinor<C> hops(Spinor<C> tp, Spinor<C> tm, Spinor<C> xp, Spinor<C> xm, C u0f,
                                 C u0b, C u1f, C u1b, R sf, R sb) {
  C h = cscale(cmul(u0f, csub(tp.s0, tp.s1)), sf);
  C s0 = h, s1 = mk<R>(-h.x, -h.y);
  h = cscale(cmulc(u0b, cadd(tm.s0, tm.s1)), sb);
  s0 = cadd(s0, h);
  s1 = cadd(s1, h);
  h = cmul(u1f, cadd(xp.s0, ctimes_i(xp.s1)));
  s0 = cadd(s0, h);
  s1 = csub(s1, ctimes_i(h));
  h = cmulc(u1b, csub(xm.s0, ctimes_i(xm.s1)));
  s0 = cadd(s0, h);
  s1 = cadd(s1, ctimes_i(h));
  return Spinor<C>{cscale(s0, R(-0.5)), cscale(s1, R(-0.5))};
}

// Periodic index for v in [-1, ...): the halo row/column -1 maps to n - 1 and n maps to 0.  Tile
// positions past n (a tile wider than a small lattice) hold no site's neighbour; they are
// clamped to 0 so that every load stays inside the field.
__device__ inline int wrap_index(int v, int n) {
  if (v < 0) return v + n;
  if (v < n) return v;
  return v - n < n ? v - n : 0;
}

// y = D x (or b - D x) on TR x TC tiles (TR * TC = 256 * SPT, SPT sites per thread, rows rr,
// rr + TR / SPT, ...): the tile and its one-site halo, rows t0 - 1 .. t0 + TR and columns
// x0 - 1 .. x0 + TC (periodic wrap), are read from HBM once into LDS; every site then takes its
// four neighbours from LDS.  Taller tiles read fewer halo rows per site.
template <int TC, int SPT, typename R, typename L, typename Vin, typename Vout>
__global__ __launch_bounds__(256) void k_wilson_apply(const L* __restrict__ U0,
                                                      const L* __restrict__ U1,
                                                      const Vin* __restrict__ x,
                                                      Vout* __restrict__ y,
                                                      const double2* __restrict__ b, int nt,
                                                      int nx, R mp2, int64_t stride,
                                                      const RhsState* __restrict__ st) {
  constexpr int TR = 256 * SPT / TC, W = TC + 2;
  using C = cplx<R>;
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  __shared__ Spinor<C> s[(TR + 2) * W];
  const int tiles_x = (nx + TC - 1) / TC;
  const int ty = blockIdx.x / tiles_x, tx = blockIdx.x - ty * tiles_x;
  const int t0 = ty * TR, x0 = tx * TC;
  const Spinor<Vin>* xr = reinterpret_cast<const Spinor<Vin>*>(x + r * stride);
  for (int e = threadIdx.x; e < (TR + 2) * W; e += 256) {
    const int rw = e / W, c = e - rw * W;
    const int tt = wrap_index(t0 + rw - 1, nt), xx = wrap_index(x0 + c - 1, nx);
    s[e] = sconv<C>(xr[int64_t(tt) * nx + xx]);
  }
  __syncthreads();
  Spinor<Vout>* yr = reinterpret_cast<Spinor<Vout>*>(y + r * stride);
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int rr = threadIdx.x / TC + q * (TR / SPT), cc = threadIdx.x % TC;
    const int t = t0 + rr, xc = x0 + cc;
    if (t >= nt || xc >= nx) continue;
    const int n = t * nx + xc;
    const int tb = t == 0 ? nt - 1 : t - 1, xb = xc == 0 ? nx - 1 : xc - 1;
    const int Ls = (rr + 1) * W + (cc + 1);
    const Spinor<C> h = hops<C, R>(s[Ls + W], s[Ls - W], s[Ls + 1], s[Ls - 1], load_link<R>(U0, n),
                                   load_link<R>(U0, int64_t(tb) * nx + xc), load_link<R>(U1, n),
                                   load_link<R>(U1, int64_t(t) * nx + xb), t == nt - 1 ? R(-1) : R(1),
                                   t == 0 ? R(-1) : R(1));
    const Spinor<C> me = s[Ls];
    Spinor<C> o{cadd(cscale(me.s0, mp2), h.s0), cadd(cscale(me.s1, mp2), h.s1)};
    if (b) {
      const Spinor<double2> bb = reinterpret_cast<const Spinor<double2>*>(b + r * stride)[n];
      const Spinor<double2> od = sconv<double2>(o);
      yr[n] = sconv<Vout>(Spinor<double2>{csub(bb.s0, od.s0), csub(bb.s1, od.s1)});
    } else {
      yr[n] = sconv<Vout>(o);
    }
  }
}

// One colour c = (t + x) mod 2 of the red-black point Gauss-Seidel sweep on D x = b:
// x(n) <- x(n) + (b(n) - (D x)(n)) / (m0 + 2) = (b(n) - hops(n)) / (m0 + 2) for n of colour c
// (the diagonal of D is (m0 + 2) I); b = null means b = 0.  Tiles of TR x TC sites
// (TR * TC = 512, t0 and x0 even) hold the 256 colour-c sites of the tile, one per thread; only
// the opposite colour, which their neighbours have, is staged in LDS: row rw of the halo
// region keeps its W / 2 opposite-colour sites, column c at slot c / 2.
template <int TC, typename R, typename L, typename Vx>
__global__ __launch_bounds__(256) void k_wilson_gs(const L* __restrict__ U0,
                                                   const L* __restrict__ U1, Vx* x,
                                                   const double2* __restrict__ b, int nt,
                                                   int nx, R inv_mp2, int colour, int64_t stride,
                                                   const RhsState* __restrict__ st) {
  constexpr int TR = 512 / TC, W = TC + 2, H = W / 2;
  using C = cplx<R>;
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  __shared__ Spinor<C> s[(TR + 2) * H];
  const int tiles_x = (nx + TC - 1) / TC;
  const int ty = blockIdx.x / tiles_x, tx = blockIdx.x - ty * tiles_x;
  const int t0 = ty * TR, x0 = tx * TC;
  Spinor<Vx>* xr = reinterpret_cast<Spinor<Vx>*>(x + r * stride);
  // halo position (rw, c) is site (t0 + rw - 1, x0 + c - 1), of colour (rw + c) mod 2
  for (int e = threadIdx.x; e < (TR + 2) * H; e += 256) {
    const int rw = e / H, j = e - rw * H;
    const int c = 2 * j + ((1 - colour + rw) & 1);
    const int tt = wrap_index(t0 + rw - 1, nt), xx = wrap_index(x0 + c - 1, nx);
    s[e] = sconv<C>(xr[int64_t(tt) * nx + xx]);
  }
  __syncthreads();
  const int rr = threadIdx.x / (TC / 2), k = threadIdx.x - rr * (TC / 2);
  const int t = t0 + rr;
  const int cc = 2 * k + ((t + colour) & 1);
  const int xc = x0 + cc;
  if (t >= nt || xc >= nx) return;
  const int n = t * nx + xc;
  const int tb = t == 0 ? nt - 1 : t - 1, xb = xc == 0 ? nx - 1 : xc - 1;
  const int R0 = rr + 1, C0 = cc + 1;
  const Spinor<C> h = hops<C, R>(s[(R0 + 1) * H + (C0 >> 1)], s[(R0 - 1) * H + (C0 >> 1)],
                                 s[R0 * H + ((C0 + 1) >> 1)], s[R0 * H + ((C0 - 1) >> 1)],
                                 load_link<R>(U0, n), load_link<R>(U0, int64_t(tb) * nx + xc),
                                 load_link<R>(U1, n), load_link<R>(U1, int64_t(t) * nx + xb),
                                 t == nt - 1 ? R(-1) : R(1), t == 0 ? R(-1) : R(1));
  Spinor<C> f{czero<R>(), czero<R>()};
  if (b) f = sconv<C>(reinterpret_cast<const Spinor<double2>*>(b + r * stride)[n]);
  xr[n] = sconv<Vx>(Spinor<C>{cscale(csub(f.s0, h.s0), inv_mp2), cscale(csub(f.s1, h.s1), inv_mp2)});
}

// NS red-black sweeps (colours 0 then 1, NS = 1 or 2) from xin into xout (distinct buffers:
// workgroups read their halos from xin while others write xout).  A workgroup owns a
// TR x TC tile and stages x on the tile plus a halo of HW = 2 NS sites and b on the tile plus
// HW - 1 sites (periodic indices) in LDS.  Half-sweep h updates the sites of its colour that are
// at least h + 1 sites inside the staged region: their neighbours there hold the values after
// half-sweep h, so every value inside the tile is exactly the per-colour sweeps' value (halo
// sites are recomputed by each workgroup that needs them, from the same inputs in the same
// order).  Only the tile is written back.
template <int NS, int TR, int TC, typename R, typename L, typename Vx>
__global__ __launch_bounds__(256) void k_wilson_gs_fused(const L* __restrict__ U0,
                                                         const L* __restrict__ U1,
                                                         const Vx* __restrict__ xin,
                                                         Vx* __restrict__ xout,
                                                         const double2* __restrict__ b, int nt,
                                                         int nx, R inv_mp2, int64_t stride,
                                                         const RhsState* __restrict__ st) {
  constexpr int HW = 2 * NS, RW = TC + 2 * HW, RH = TR + 2 * HW, BW = RW - 2, BH = RH - 2;
  using C = cplx<R>;
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  __shared__ Spinor<C> xs[RH * RW];
  __shared__ Spinor<C> bs[BH * BW];
  const int tiles_x = (nx + TC - 1) / TC;
  const int ty = blockIdx.x / tiles_x, tx = blockIdx.x - ty * tiles_x;
  const int t0 = ty * TR - HW, x0 = tx * TC - HW;   // region origin (global, may be negative)
  const Spinor<Vx>* xr = reinterpret_cast<const Spinor<Vx>*>(xin + r * stride);
  Spinor<Vx>* xw = reinterpret_cast<Spinor<Vx>*>(xout + r * stride);
  // staging with several loads in flight per thread (see stage())
  stage<4, 256, Spinor<Vx>>(RH * RW, [&](int e) {
    const int rw = e / RW, c = e - rw * RW;
    const int tt = ((t0 + rw) % nt + nt) % nt, xx = ((x0 + c) % nx + nx) % nx;
    return xr[int64_t(tt) * nx + xx];
  }, [&](int e, Spinor<Vx> v) { xs[e] = sconv<C>(v); });
  if (b) {
    const Spinor<double2>* br = reinterpret_cast<const Spinor<double2>*>(b + r * stride);
    stage<4, 256, Spinor<double2>>(BH * BW, [&](int e) {
      const int rw = e / BW, c = e - rw * BW;
      const int tt = ((t0 + 1 + rw) % nt + nt) % nt, xx = ((x0 + 1 + c) % nx + nx) % nx;
      return br[int64_t(tt) * nx + xx];
    }, [&](int e, Spinor<double2> v) { bs[e] = sconv<C>(v); });
  } else {
    for (int e = threadIdx.x; e < BH * BW; e += 256) bs[e] = Spinor<C>{czero<R>(), czero<R>()};
  }
  __syncthreads();
  for (int hs = 0; hs < 2 * NS; ++hs) {
    const int colour = hs & 1, lo = hs + 1;
    const int rows = RH - 2 * lo, pairs = (RW - 2 * lo) / 2;   // RW - 2 lo is even
    // region parity: t0 + x0 is even, so site (rw, c) has colour (rw + c) mod 2
    for (int e = threadIdx.x; e < rows * pairs; e += 256) {
      const int rw = lo + e / pairs;
      const int c = lo + 2 * (e - (e / pairs) * pairs) + ((rw + lo + colour) & 1);
      const int t = ((t0 + rw) % nt + nt) % nt, xc = ((x0 + c) % nx + nx) % nx;
      const int n = t * nx + xc;
      const int tb = t == 0 ? nt - 1 : t - 1, xb = xc == 0 ? nx - 1 : xc - 1;
      const int q = rw * RW + c;
      const Spinor<C> h = hops<C, R>(xs[q + RW], xs[q - RW], xs[q + 1], xs[q - 1], load_link<R>(U0, n),
                                     load_link<R>(U0, int64_t(tb) * nx + xc), load_link<R>(U1, n),
                                     load_link<R>(U1, int64_t(t) * nx + xb), t == nt - 1 ? R(-1) : R(1),
                                     t == 0 ? R(-1) : R(1));
      const Spinor<C> f = bs[(rw - 1) * BW + (c - 1)];
      xs[q] = Spinor<C>{cscale(csub(f.s0, h.s0), inv_mp2), cscale(csub(f.s1, h.s1), inv_mp2)};
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < TR * TC; e += 256) {
    const int rr = e / TC, cc = e - rr * TC;
    const int t = ty * TR + rr, xc = tx * TC + cc;
    if (t >= nt || xc >= nx) continue;
    const Spinor<C> v = xs[(rr + HW) * RW + (cc + HW)];
    xw[int64_t(t) * nx + xc] = Spinor<Vx>{cconv<Vx>(v.s0), cconv<Vx>(v.s1)};
  }
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


template <typename R, typename L, typename Vin, typename Vout>
static void wilson_apply_t(hipStream_t s, const void* U0, const void* U1, const void* x, void* y,
                           const double2* b, int nt, int nx, double m0, int nrhs, int64_t stride,
                           const RhsState* st) {
  if (nx >= 64) {
    // FP32: 8 x 64 tiles, two sites per thread (5.68 against 5.33 TB/s at 4096^2, fewer halo
    // rows); FP64: 4 x 64 (two sites per thread measured 5.53 against 5.71 TB/s)
    constexpr int SPT = sizeof(R) == 4 ? 2 : 1;
    dim3 g(unsigned(((nx + 63) / 64) * ((nt + 4 * SPT - 1) / (4 * SPT))), unsigned(nrhs));
    AMAMG_LAUNCH((k_wilson_apply<64, SPT, R, L, Vin, Vout>), g, dim3(256), 0, s, (const L*)U0,
                       (const L*)U1, (const Vin*)x, (Vout*)y, b, nt, nx, R(m0 + 2.0), stride, st);
  } else {
    dim3 g(unsigned(((nx + 15) / 16) * ((nt + 15) / 16)), unsigned(nrhs));
    AMAMG_LAUNCH((k_wilson_apply<16, 1, R, L, Vin, Vout>), g, dim3(256), 0, s, (const L*)U0,
                       (const L*)U1, (const Vin*)x, (Vout*)y, b, nt, nx, R(m0 + 2.0), stride, st);
  }
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
  if (nx >= 64) {
    dim3 g(unsigned(((nx + 63) / 64) * ((nt + 7) / 8)), unsigned(nrhs));
    AMAMG_LAUNCH((k_wilson_gs<64, R, L, Vx>), g, dim3(256), 0, s, (const L*)U0, (const L*)U1,
                       (Vx*)x, b, nt, nx, R(1.0 / (m0 + 2.0)), colour, stride, st);
  } else {
    dim3 g(unsigned(((nx + 15) / 16) * ((nt + 31) / 32)), unsigned(nrhs));
    AMAMG_LAUNCH((k_wilson_gs<16, R, L, Vx>), g, dim3(256), 0, s, (const L*)U0, (const L*)U1,
                       (Vx*)x, b, nt, nx, R(1.0 / (m0 + 2.0)), colour, stride, st);
  }
}

void wilson_gs(hipStream_t s, LinkStore ls, const void* U0, const void* U1, Real vx, void* x,
               const double2* b, int nt, int nx, double m0, int colour, int nrhs, int64_t stride,
               const RhsState* st) {
  if (ls == LINK_F64 && vx == F64) wilson_gs_t<double, double2, double2>(s, U0, U1, x, b, nt, nx, m0, colour, nrhs, stride, st);
  else if (ls == LINK_F32) wilson_gs_t<float, float2, float2>(s, U0, U1, x, b, nt, nx, m0, colour, nrhs, stride, st);
  else wilson_gs_t<float, bf16c, float2>(s, U0, U1, x, b, nt, nx, m0, colour, nrhs, stride, st);
}

// Tile widths of the fused smoother (16 rows each): every site's update is the same arithmetic
// whatever the tile, so the width is a free launch parameter.  FP64 stops at 32 columns for the
// LDS budget.  tc = 0 takes the default: the widest that fits the lattice.
template <typename R> constexpr int fused_max_tc() { return sizeof(R) == 4 ? 64 : 32; }

template <int NS, typename R, typename L, typename Vx>
static void wilson_gs_fused_t(hipStream_t s, const void* U0, const void* U1, const void* xin, void* x,
                              const double2* b, int nt, int nx, double m0, int nrhs, int64_t stride,
                              const RhsState* st, int tc) {
  if (tc == 0) tc = nx >= fused_max_tc<R>() ? fused_max_tc<R>() : 16;
  if (tc > fused_max_tc<R>() || nx < tc) tc = 16;
  const R inv = R(1.0 / (m0 + 2.0));
  dim3 g(unsigned(((nx + tc - 1) / tc) * ((nt + 15) / 16)), unsigned(nrhs));
  if (tc == 64) {
    if constexpr (fused_max_tc<R>() >= 64)
      AMAMG_LAUNCH((k_wilson_gs_fused<NS, 16, 64, R, L, Vx>), g, dim3(256), 0, s, (const L*)U0, (const L*)U1,
                   (const Vx*)xin, (Vx*)x, b, nt, nx, inv, stride, st);
  } else if (tc == 32) {
    AMAMG_LAUNCH((k_wilson_gs_fused<NS, 16, 32, R, L, Vx>), g, dim3(256), 0, s, (const L*)U0, (const L*)U1,
                 (const Vx*)xin, (Vx*)x, b, nt, nx, inv, stride, st);
  } else {
    AMAMG_LAUNCH((k_wilson_gs_fused<NS, 16, 16, R, L, Vx>), g, dim3(256), 0, s, (const L*)U0, (const L*)U1,
                 (const Vx*)xin, (Vx*)x, b, nt, nx, inv, stride, st);
  }
}

void wilson_gs_sweeps(hipStream_t s, LinkStore ls, const void* U0, const void* U1, Real vx, const void* xin,
                      void* x, const double2* b, int nt, int nx, double m0, int sweeps, int nrhs,
                      int64_t stride, const RhsState* st, int tc) {
  if (sweeps == 2) {
    if (ls == LINK_F64 && vx == F64) wilson_gs_fused_t<2, double, double2, double2>(s, U0, U1, xin, x, b, nt, nx, m0, nrhs, stride, st, tc);
    else if (ls == LINK_F32) wilson_gs_fused_t<2, float, float2, float2>(s, U0, U1, xin, x, b, nt, nx, m0, nrhs, stride, st, tc);
    else wilson_gs_fused_t<2, float, bf16c, float2>(s, U0, U1, xin, x, b, nt, nx, m0, nrhs, stride, st, tc);
  } else {
    if (ls == LINK_F64 && vx == F64) wilson_gs_fused_t<1, double, double2, double2>(s, U0, U1, xin, x, b, nt, nx, m0, nrhs, stride, st, tc);
    else if (ls == LINK_F32) wilson_gs_fused_t<1, float, float2, float2>(s, U0, U1, xin, x, b, nt, nx, m0, nrhs, stride, st, tc);
    else wilson_gs_fused_t<1, float, bf16c, float2>(s, U0, U1, xin, x, b, nt, nx, m0, nrhs, stride, st, tc);
  }
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
