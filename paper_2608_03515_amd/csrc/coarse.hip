// Coarse-level kernels: block-stencil apply (Galerkin operator P^H A P, paper's Multilevel
// approach section), its 16-colour point-block Gauss-Seidel sweep, and the dense coarsest solve.
//
// A coarse operator is stored as a 5 x 5 block stencil: node n couples to n + (dt, dx),
// dt, dx in [-2, 2], through a b x b complex block A[n][(dt+2)*5 + (dx+2)][i][j] (node-major:
// everything a node needs is contiguous).  Coarse vectors are [rhs][node][b] complex.
//
// Lane layout (block size B a power of two, B <= 64): the lanes of one node cover its B rows,
// LJ lanes per row; lane (i, jl) handles columns jl, jl + LJ, ...  With B*B <= 64 one wave
// holds 64 / (B*B) nodes and reads whole B x B blocks per offset in one coalesced access;
// otherwise one node per wave.  Row sums are finished with xor shuffles inside the LJ lanes.
#include <type_traits>

#include "launch.hpp"

namespace amamg {

template <int B> struct Lanes {
  static constexpr int LJ = (B * B <= 64) ? B : 64 / B;     // lanes per row
  static constexpr int CPL = B / LJ;                        // columns per lane
  static constexpr int LPN = B * LJ;                        // lanes per node
  static constexpr int NPW = 64 / LPN;                      // nodes per wave
  static constexpr int NPB = 4 * NPW;                       // nodes per 256-thread block
};

__device__ inline int wrap1(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

template <int LJ, typename R> __device__ inline R group_sum(R v) {
#pragma unroll
  for (int off = LJ >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// y[n] = sum_d A[n][d] x[n+d]   (or f - that)
template <int B, typename R, typename M, typename Vin, typename Vout>
__global__ __launch_bounds__(256) void k_stencil_apply(const M* __restrict__ A,
                                                       const Vin* __restrict__ x,
                                                       Vout* __restrict__ y,
                                                       const Vout* __restrict__ f, int Lt, int Lx,
                                                       int64_t stride,
                                                       const RhsState* __restrict__ st) {
  using Ly = Lanes<B>;
  using C = cplx<R>;
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int slot = lane / Ly::LPN, i = (lane / Ly::LJ) % B, jl = lane % Ly::LJ;
  const int n = (xcd_block(blockIdx.x, gridDim.x) * 4 + wv) * Ly::NPW + slot;
  const bool live = n < Lt * Lx;
  const int nn = live ? n : 0;
  const int t = nn / Lx, xc = nn - t * Lx;
  const Vin* xr = x + r * stride;
  const M* An = A + int64_t(nn) * 25 * B * B + i * B;
  C acc = czero<R>();
#pragma unroll
  for (int dt = -2; dt <= 2; ++dt) {
    const int tt = wrap1(t + dt, Lt) * Lx;
#pragma unroll
    for (int dx = -2; dx <= 2; ++dx) {
      const int m = tt + wrap1(xc + dx, Lx);
      const M* blk = An + ((dt + 2) * 5 + (dx + 2)) * B * B;
      const Vin* xm = xr + int64_t(m) * B;
#pragma unroll
      for (int c = 0; c < Ly::CPL; ++c) {
        const int j = jl + Ly::LJ * c;
        acc = cfma(cconv<C>(blk[j]), cconv<C>(xm[j]), acc);
      }
    }
  }
  acc.x = group_sum<Ly::LJ>(acc.x);
  acc.y = group_sum<Ly::LJ>(acc.y);
  if (live && jl == 0) {
    const int64_t o = r * stride + int64_t(n) * B + i;
    if (f) acc = csub(cconv<C>(f[o]), acc);
    y[o] = cconv<Vout>(acc);
  }
}

// Colour c = (I mod 4) * 4 + (J mod 4); nodes of one colour do not couple (stencil reach 2).
// x_n <- Dinv_n (f_n - sum_{d != 0} A_nd x_{n+d})  (equals x_n + Dinv_n (f - A x)_n).
template <int B, typename R, typename M, typename Vx>
__global__ __launch_bounds__(256) void k_stencil_gs(const M* __restrict__ A,
                                                    const M* __restrict__ Dinv, Vx* x,
                                                    const Vx* __restrict__ f, int Lt, int Lx,
                                                    int colour, int64_t stride,
                                                    const RhsState* __restrict__ st) {
  using Ly = Lanes<B>;
  using C = cplx<R>;
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int slot = lane / Ly::LPN, i = (lane / Ly::LJ) % B, jl = lane % Ly::LJ;
  const int k = (blockIdx.x * 4 + wv) * Ly::NPW + slot;
  const int qx = Lx >> 2;
  const int ncn = (Lt >> 2) * qx;
  const bool live = k < ncn;
  const int kk = live ? k : 0;
  const int t = 4 * (kk / qx) + (colour >> 2), xc = 4 * (kk % qx) + (colour & 3);
  const int n = t * Lx + xc;
  Vx* xr = x + r * stride;
  const M* An = A + int64_t(n) * 25 * B * B + i * B;
  C acc = czero<R>();
#pragma unroll
  for (int dt = -2; dt <= 2; ++dt) {
    const int tt = wrap1(t + dt, Lt) * Lx;
#pragma unroll
    for (int dx = -2; dx <= 2; ++dx) {
      if (dt == 0 && dx == 0) continue;
      const int m = tt + wrap1(xc + dx, Lx);
      const M* blk = An + ((dt + 2) * 5 + (dx + 2)) * B * B;
      const Vx* xm = xr + int64_t(m) * B;
#pragma unroll
      for (int c = 0; c < Ly::CPL; ++c) {
        const int j = jl + Ly::LJ * c;
        acc = cfma(cconv<C>(blk[j]), cconv<C>(xm[j]), acc);
      }
    }
  }
  acc.x = group_sum<Ly::LJ>(acc.x);
  acc.y = group_sum<Ly::LJ>(acc.y);
  C res = acc;
  res.x = -res.x;
  res.y = -res.y;
  if (f && live) res = cadd(res, cconv<C>(f[r * stride + int64_t(n) * B + i]));
  // x_n[i] = sum_j Dinv[n][i][j] res_j; res_j sits in every lane of row j of this node
  const int node_lane0 = slot * Ly::LPN;
  const M* Dn = Dinv + int64_t(n) * B * B + i * B;
  C out = czero<R>();
#pragma unroll
  for (int c = 0; c < Ly::CPL; ++c) {
    const int j = jl + Ly::LJ * c;
    const R re = __shfl(res.x, node_lane0 + j * Ly::LJ), im = __shfl(res.y, node_lane0 + j * Ly::LJ);
    out = cfma(cconv<C>(Dn[j]), mk<R>(re, im), out);
  }
  out.x = group_sum<Ly::LJ>(out.x);
  out.y = group_sum<Ly::LJ>(out.y);
  if (live && jl == 0) xr[int64_t(n) * B + i] = cconv<Vx>(out);
}

// One node's Gauss-Seidel update x_n <- Dinv_n (f_n - sum_{d != 0} A_nd x_{n+d}) for the lanes of
// that node (the arithmetic of k_stencil_gs), returning out = row i of the new x_n (summed over
// the node's lanes).  With sub >= 0 the neighbour at offset (0, -1) is taken from `sub_val`
// (this lane's columns of it) instead of memory.
template <int B, typename R, typename M, typename Vx>
__device__ inline cplx<R> gs_node(const M* __restrict__ A, const M* __restrict__ Dinv, const Vx* xr,
                                  const Vx* __restrict__ fr, int Lt, int Lx, int t, int xc, int i, int jl,
                                  int node_lane0, bool live, bool sub, const cplx<R>* sub_val) {
  using Ly = Lanes<B>;
  using C = cplx<R>;
  const int n = t * Lx + xc;
  const M* An = A + int64_t(n) * 25 * B * B + i * B;
  C acc = czero<R>();
#pragma unroll
  for (int dt = -2; dt <= 2; ++dt) {
    const int tt = wrap1(t + dt, Lt) * Lx;
#pragma unroll
    for (int dx = -2; dx <= 2; ++dx) {
      if (dt == 0 && dx == 0) continue;
      const int m = tt + wrap1(xc + dx, Lx);
      const M* blk = An + ((dt + 2) * 5 + (dx + 2)) * B * B;
      const Vx* xm = xr + int64_t(m) * B;
#pragma unroll
      for (int c = 0; c < Ly::CPL; ++c) {
        const int j = jl + Ly::LJ * c;
        const C xv = (sub && dt == 0 && dx == -1) ? sub_val[c] : cconv<C>(xm[j]);
        acc = cfma(cconv<C>(blk[j]), xv, acc);
      }
    }
  }
  acc.x = group_sum<Ly::LJ>(acc.x);
  acc.y = group_sum<Ly::LJ>(acc.y);
  C res = acc;
  res.x = -res.x;
  res.y = -res.y;
  if (fr && live) res = cadd(res, cconv<C>(fr[int64_t(n) * B + i]));
  const M* Dn = Dinv + int64_t(n) * B * B + i * B;
  C out = czero<R>();
#pragma unroll
  for (int c = 0; c < Ly::CPL; ++c) {
    const int j = jl + Ly::LJ * c;
    const R re = __shfl(res.x, node_lane0 + j * Ly::LJ), im = __shfl(res.y, node_lane0 + j * Ly::LJ);
    out = cfma(cconv<C>(Dn[j]), mk<R>(re, im), out);
  }
  out.x = group_sum<Ly::LJ>(out.x);
  out.y = group_sum<Ly::LJ>(out.y);
  return out;
}

// Colours c0 = 4 a + 2 q and c0 + 1 in one launch, exactly as two k_stencil_gs launches.  Node
// (I, J) of colour c0 + 1 and node (I, J - 1) of colour c0 pair up one to one, and within the
// stencil reach (2) each member of a pair couples to no other node of the two colours but its
// partner.  One wave per pair updates (I, J - 1) from the values before the launch, writes it,
// then updates (I, J) with that new value at offset (0, -1) and the values before the launch
// elsewhere: no other wave reads or writes either node.
template <int B, typename R, typename M, typename Vx>
__global__ __launch_bounds__(256) void k_stencil_gs_pair(const M* __restrict__ A,
                                                         const M* __restrict__ Dinv, Vx* x,
                                                         const Vx* __restrict__ f, int Lt, int Lx,
                                                         int c0, int64_t stride,
                                                         const RhsState* __restrict__ st) {
  using Ly = Lanes<B>;
  using C = cplx<R>;
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int slot = lane / Ly::LPN, i = (lane / Ly::LJ) % B, jl = lane % Ly::LJ;
  const int qx = Lx >> 2;
  const int ncn = (Lt >> 2) * qx;
  const int k = (blockIdx.x * 4 + wv) * Ly::NPW + slot;
  const bool live = k < ncn;
  const int kk = live ? k : 0;
  const int colour = c0 + 1;
  const int t = 4 * (kk / qx) + (colour >> 2), xc = 4 * (kk % qx) + (colour & 3);   // xc >= 1
  Vx* xr = x + r * stride;
  const Vx* fr = f ? f + r * stride : nullptr;
  const int node_lane0 = slot * Ly::LPN;
  C sub_val[Ly::CPL];
  const C v = gs_node<B, R, M, Vx>(A, Dinv, xr, fr, Lt, Lx, t, xc - 1, i, jl, node_lane0, live, false, sub_val);
  if (live && jl == 0) xr[int64_t(t * Lx + xc - 1) * B + i] = cconv<Vx>(v);
#pragma unroll
  for (int c = 0; c < Ly::CPL; ++c) {
    const int j = jl + Ly::LJ * c;
    // the partner's new value in the storage type, as the two-launch sequence reads it
    const R re = __shfl(v.x, node_lane0 + j * Ly::LJ), im = __shfl(v.y, node_lane0 + j * Ly::LJ);
    sub_val[c] = cconv<C>(cconv<Vx>(mk<R>(re, im)));
  }
  const C out = gs_node<B, R, M, Vx>(A, Dinv, xr, fr, Lt, Lx, t, xc, i, jl, node_lane0, live, true, sub_val);
  if (live && jl == 0) xr[int64_t(t * Lx + xc) * B + i] = cconv<Vx>(out);
}

// k_stencil_gs_pair for B = 8 (one node per wave, lane (i, j) = row i, column j) over RB
// right-hand sides per wave: the wave loads both nodes' 24 neighbour blocks and inverse diagonal
// blocks once into registers and runs its right-hand sides through them, so the operator is read
// once per RB right-hand sides.  Per right-hand side all neighbour values of both nodes are
// loaded before the first node is written (the second node's only coupling to the first is the
// partner at (0, -1), which comes from the first node's new value); the arithmetic and its order
// are those of k_stencil_gs_pair, so the results are bitwise the same.
template <int RB, typename R, typename M, typename Vx>
__global__ __launch_bounds__(256) void k_stencil_gs_pair_mr(const M* __restrict__ A,
                                                            const M* __restrict__ Dinv, Vx* x,
                                                            const Vx* __restrict__ f, int Lt, int Lx,
                                                            int c0, int nrhs, int64_t stride,
                                                            const RhsState* __restrict__ st) {
  constexpr int B = 8, NB = 24;
  using C = cplx<R>;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = lane >> 3, jl = lane & 7;
  const int qx = Lx >> 2, ncn = (Lt >> 2) * qx;
  const int k = blockIdx.x * 4 + wv;
  if (k >= ncn) return;                       // whole waves; the kernel has no block barrier
  const int colour = c0 + 1;
  const int t = 4 * (k / qx) + (colour >> 2), xc = 4 * (k % qx) + (colour & 3);   // xc >= 1
  const int n1 = t * Lx + xc - 1, n2 = t * Lx + xc;
  int m1[NB], m2[NB];
  C a1[NB], a2[NB];
  {
    int q = 0;
#pragma unroll
    for (int dt = -2; dt <= 2; ++dt) {
      const int tt = wrap1(t + dt, Lt) * Lx;
#pragma unroll
      for (int dx = -2; dx <= 2; ++dx) {
        if (dt == 0 && dx == 0) continue;
        const int d = (dt + 2) * 5 + (dx + 2);
        m1[q] = tt + wrap1(xc - 1 + dx, Lx);
        m2[q] = tt + wrap1(xc + dx, Lx);
        a1[q] = cconv<C>(A[(int64_t(n1) * 25 + d) * B * B + i * B + jl]);
        a2[q] = cconv<C>(A[(int64_t(n2) * 25 + d) * B * B + i * B + jl]);
        ++q;
      }
    }
  }
  const C d1 = cconv<C>(Dinv[int64_t(n1) * B * B + i * B + jl]);
  const C d2 = cconv<C>(Dinv[int64_t(n2) * B * B + i * B + jl]);
  constexpr int PARTNER = 2 * 5 + 1;          // index q of offset (0, -1): rows dt = -2, -1 (q 0..9), then dx = -2 (q 10)
  const int r0 = blockIdx.y * RB;
  for (int rr = 0; rr < RB; ++rr) {
    const int r = r0 + rr;
    if (r >= nrhs) break;
    if (st && !st[r].active) continue;
    Vx* xr = x + r * stride;
    C v1[NB], v2[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      v1[q] = cconv<C>(xr[int64_t(m1[q]) * B + jl]);
      if (q != PARTNER) v2[q] = cconv<C>(xr[int64_t(m2[q]) * B + jl]);
    }
    const C f1 = f ? cconv<C>(f[r * stride + int64_t(n1) * B + i]) : czero<R>();
    const C f2 = f ? cconv<C>(f[r * stride + int64_t(n2) * B + i]) : czero<R>();
    // first node
    C acc = czero<R>();
#pragma unroll
    for (int q = 0; q < NB; ++q) acc = cfma(a1[q], v1[q], acc);
    acc.x = group_sum<8>(acc.x);
    acc.y = group_sum<8>(acc.y);
    C res = mk<R>(-acc.x, -acc.y);
    if (f) res = cadd(res, f1);
    C out = cfma(d1, mk<R>(__shfl(res.x, jl * 8), __shfl(res.y, jl * 8)), czero<R>());
    out.x = group_sum<8>(out.x);
    out.y = group_sum<8>(out.y);
    if (jl == 0) xr[int64_t(n1) * B + i] = cconv<Vx>(out);
    // the partner's new value in the storage type, as the two-launch sequence reads it
    v2[PARTNER] = cconv<C>(cconv<Vx>(mk<R>(__shfl(out.x, jl * 8), __shfl(out.y, jl * 8))));
    // second node
    acc = czero<R>();
#pragma unroll
    for (int q = 0; q < NB; ++q) acc = cfma(a2[q], v2[q], acc);
    acc.x = group_sum<8>(acc.x);
    acc.y = group_sum<8>(acc.y);
    res = mk<R>(-acc.x, -acc.y);
    if (f) res = cadd(res, f2);
    out = cfma(d2, mk<R>(__shfl(res.x, jl * 8), __shfl(res.y, jl * 8)), czero<R>());
    out.x = group_sum<8>(out.x);
    out.y = group_sum<8>(out.y);
    if (jl == 0) xr[int64_t(n2) * B + i] = cconv<Vx>(out);
  }
}

// One colour block qb of the coarse sweep (coarse_colour(4 qb) .. coarse_colour(4 qb + 3)) for
// B = 8 in one launch: the block's nodes form 2 x 2 groups (rows I0, I0 + 1, columns J0, J0 + 1)
// that do not couple with each other, and the four updates of a group run in colour order.  Two
// waves per group: the lower wave updates (I0, J0) then (I0, J0 + 1) exactly as
// k_stencil_gs_pair_mr does, and leaves their new values (in the storage type, as a launch per
// colour pair would read them) in LDS; the upper wave then updates (I0 + 1, J0) and (I0 + 1,
// J0 + 1) with those values for its in-group neighbours above.  Per right-hand side the upper
// wave runs one phase behind the lower one; every thread passes the same RB + 1 barriers.
// The results are bitwise those of the two colour-pair launches.
template <int RB, typename R, typename M, typename Vx>
__global__ __launch_bounds__(256) void k_stencil_gs_quad_mr(const M* __restrict__ A,
                                                            const M* __restrict__ Dinv, Vx* x,
                                                            const Vx* __restrict__ f, int Lt, int Lx,
                                                            int qb, int nrhs, int64_t stride,
                                                            const RhsState* __restrict__ st) {
  constexpr int B = 8, NB = 24;
  // neighbour slots (loop order dt, dx = -2..2 without (0, 0)) of the in-group offsets
  constexpr int UPL = 6, UP = 7, UPR = 8, LEFT = 11;   // (-1,-1), (-1,0), (-1,+1), (0,-1)
  using C = cplx<R>;
  __shared__ C lower[2][RB][2][B];                    // [group slot][rhs][node][row]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = lane >> 3, jl = lane & 7;
  const int gs = wv >> 1, hi = wv & 1;
  const int qx = Lx >> 2, ngr = (Lt >> 2) * qx;
  const int k = blockIdx.x * 2 + gs;
  const bool valid = k < ngr;
  const int kk = valid ? k : 0;
  const int t = 4 * (kk / qx) + 2 * (qb >> 1) + hi, xc = 4 * (kk % qx) + 2 * (qb & 1);
  const int n1 = t * Lx + xc, n2 = n1 + 1;
  int m1[NB], m2[NB];
  C a1[NB], a2[NB];
  {
    int q = 0;
#pragma unroll
    for (int dt = -2; dt <= 2; ++dt) {
      const int tt = wrap1(t + dt, Lt) * Lx;
#pragma unroll
      for (int dx = -2; dx <= 2; ++dx) {
        if (dt == 0 && dx == 0) continue;
        const int d = (dt + 2) * 5 + (dx + 2);
        m1[q] = tt + wrap1(xc + dx, Lx);
        m2[q] = tt + wrap1(xc + 1 + dx, Lx);
        a1[q] = cconv<C>(A[(int64_t(n1) * 25 + d) * B * B + i * B + jl]);
        a2[q] = cconv<C>(A[(int64_t(n2) * 25 + d) * B * B + i * B + jl]);
        ++q;
      }
    }
  }
  const C d1 = cconv<C>(Dinv[int64_t(n1) * B * B + i * B + jl]);
  const C d2 = cconv<C>(Dinv[int64_t(n2) * B * B + i * B + jl]);
  const int r0 = blockIdx.y * RB;
  for (int ph = 0; ph <= RB; ++ph) {
    const int rr = ph - hi;
    const int r = r0 + rr;
    const bool work = valid && rr >= 0 && rr < RB && r < nrhs && (!st || st[r].active);
    if (work) {
      Vx* xr = x + r * stride;
      C v1[NB], v2[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const bool up1 = hi && (q == UP || q == UPR);
        const bool up2 = hi && (q == UPL || q == UP);
        if (!up1) v1[q] = cconv<C>(xr[int64_t(m1[q]) * B + jl]);
        if (!up2 && q != LEFT) v2[q] = cconv<C>(xr[int64_t(m2[q]) * B + jl]);
      }
      if (hi) {
        v1[UP] = lower[gs][rr][0][jl];
        v1[UPR] = lower[gs][rr][1][jl];
        v2[UPL] = lower[gs][rr][0][jl];
        v2[UP] = lower[gs][rr][1][jl];
      }
      const C f1 = f ? cconv<C>(f[r * stride + int64_t(n1) * B + i]) : czero<R>();
      const C f2 = f ? cconv<C>(f[r * stride + int64_t(n2) * B + i]) : czero<R>();
      C acc = czero<R>();
#pragma unroll
      for (int q = 0; q < NB; ++q) acc = cfma(a1[q], v1[q], acc);
      acc.x = group_sum<8>(acc.x);
      acc.y = group_sum<8>(acc.y);
      C res = mk<R>(-acc.x, -acc.y);
      if (f) res = cadd(res, f1);
      C out = cfma(d1, mk<R>(__shfl(res.x, jl * 8), __shfl(res.y, jl * 8)), czero<R>());
      out.x = group_sum<8>(out.x);
      out.y = group_sum<8>(out.y);
      if (jl == 0) {
        xr[int64_t(n1) * B + i] = cconv<Vx>(out);
        if (!hi) lower[gs][rr][0][i] = cconv<C>(cconv<Vx>(out));
      }
      v2[LEFT] = cconv<C>(cconv<Vx>(mk<R>(__shfl(out.x, jl * 8), __shfl(out.y, jl * 8))));
      acc = czero<R>();
#pragma unroll
      for (int q = 0; q < NB; ++q) acc = cfma(a2[q], v2[q], acc);
      acc.x = group_sum<8>(acc.x);
      acc.y = group_sum<8>(acc.y);
      res = mk<R>(-acc.x, -acc.y);
      if (f) res = cadd(res, f2);
      out = cfma(d2, mk<R>(__shfl(res.x, jl * 8), __shfl(res.y, jl * 8)), czero<R>());
      out.x = group_sum<8>(out.x);
      out.y = group_sum<8>(out.y);
      if (jl == 0) {
        xr[int64_t(n2) * B + i] = cconv<Vx>(out);
        if (!hi) lower[gs][rr][1][i] = cconv<C>(cconv<Vx>(out));
      }
    }
    __syncthreads();
  }
}

// One colour block qb of the coarse sweep for B = 8, one wave per node: a workgroup takes one
// 2 x 2 group and one right-hand side, wave v node v of the group in sweep order (I0, J0),
// (I0, J0 + 1), (I0 + 1, J0), (I0 + 1, J0 + 1).  Every wave loads its node's 24 stencil blocks,
// the inverse diagonal block and the neighbour values that this launch does not change before
// the first barrier; then the nodes update in order, one per phase, each taking the earlier
// nodes' new values (in the storage type) from LDS.  Per node the arithmetic is exactly
// k_stencil_gs_quad_mr's, so the results are bitwise the same.  With few right-hand sides this
// spreads a colour block over four times as many waves, each with a quarter of the loads.
template <typename R, typename M, typename Vx>
__global__ __launch_bounds__(256) void k_stencil_gs_node4(const M* __restrict__ A, const M* __restrict__ Dinv,
                                                          Vx* x, const Vx* __restrict__ f, int Lt, int Lx,
                                                          int qb, int nrhs, int64_t stride,
                                                          const RhsState* __restrict__ st) {
  constexpr int B = 8, NB = 24;
  constexpr int UPL = 6, UP = 7, UPR = 8, LEFT = 11;   // slots of (-1,-1), (-1,0), (-1,+1), (0,-1)
  using C = cplx<R>;
  __shared__ C fresh[3][B];                            // new values of nodes 0..2
  const int r = blockIdx.y;
  if (st && !st[r].active) return;                     // uniform over the workgroup
  const int lane = threadIdx.x & 63, v = threadIdx.x >> 6;
  const int i = lane >> 3, jl = lane & 7;
  const int qx = Lx >> 2, k = blockIdx.x;
  const int t = 4 * (k / qx) + 2 * (qb >> 1) + (v >> 1), xc = 4 * (k % qx) + 2 * (qb & 1) + (v & 1);
  const int n = t * Lx + xc;
  Vx* xr = x + r * stride;
  C a[NB], xv[NB];
  {
    int q = 0;
#pragma unroll
    for (int dt = -2; dt <= 2; ++dt) {
      const int tt = wrap1(t + dt, Lt) * Lx;
#pragma unroll
      for (int dx = -2; dx <= 2; ++dx) {
        if (dt == 0 && dx == 0) continue;
        const int d = (dt + 2) * 5 + (dx + 2);
        a[q] = cconv<C>(A[(int64_t(n) * 25 + d) * B * B + i * B + jl]);
        // the group's earlier nodes are loaded too (old values) and replaced before use
        xv[q] = cconv<C>(xr[int64_t(tt + wrap1(xc + dx, Lx)) * B + jl]);
        ++q;
      }
    }
  }
  const C d = cconv<C>(Dinv[int64_t(n) * B * B + i * B + jl]);
  const C fv = f ? cconv<C>(f[r * stride + int64_t(n) * B + i]) : czero<R>();
  __syncthreads();                                     // every load of the launch precedes every store
  for (int ph = 0; ph < 4; ++ph) {
    if (v == ph) {
      // stencil slots of the group's earlier nodes
      if (v == 1) {
        xv[LEFT] = fresh[0][jl];
      } else if (v == 2) {
        xv[UP] = fresh[0][jl];
        xv[UPR] = fresh[1][jl];
      } else if (v == 3) {
        xv[UPL] = fresh[0][jl];
        xv[UP] = fresh[1][jl];
        xv[LEFT] = fresh[2][jl];
      }
      C acc = czero<R>();
#pragma unroll
      for (int q = 0; q < NB; ++q) acc = cfma(a[q], xv[q], acc);
      acc.x = group_sum<8>(acc.x);
      acc.y = group_sum<8>(acc.y);
      C res = mk<R>(-acc.x, -acc.y);
      if (f) res = cadd(res, fv);
      C out = cfma(d, mk<R>(__shfl(res.x, jl * 8), __shfl(res.y, jl * 8)), czero<R>());
      out.x = group_sum<8>(out.x);
      out.y = group_sum<8>(out.y);
      if (jl == 0) {
        xr[int64_t(n) * B + i] = cconv<Vx>(out);
        if (v < 3) fresh[v][i] = cconv<C>(cconv<Vx>(out));
      }
    }
    if (ph < 3) __syncthreads();
  }
}

// One colour block qb of the coarse sweep for FP32 8 x 8 blocks on matrix cores.  A workgroup
// takes one 2 x 2 group of the block and a tile of 16 right-hand sides; wave v owns node v of
// the group in sweep order (I0, J0), (I0, J0 + 1), (I0 + 1, J0),
// (I0 + 1, J0 + 1).  An 8 x 8 complex block product for 16 right-hand sides is one real 16 x 16
// product, [Re y; Im y] = [[Re A, -Im A], [Im A, Re A]] [Re x; Im x], in four
// v_mfma_f32_16x16x4f32 steps (lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[4 (l / 16) + i][l % 16]).  Phase 1, all waves at once: a wave sums its node's neighbour
// blocks whose values this launch does not change (all but the group's earlier nodes), even and
// odd stencil offsets in two accumulators added at the end.  Phase 2, node by node: the owning
// wave adds the earlier nodes' new values (stencil order) from LDS, forms f - sum and applies
// the inverse diagonal block; the new values stay in LDS for the later nodes and are stored at
// the end.  The groups of a colour block do not couple, and every value read from memory is
// read before any store of the launch.  A right-hand side's arithmetic does not depend on the
// other columns of its tile, so results are the same in every batch and for every NB.
typedef float gs_mf4 __attribute__((ext_vector_type(4)));
__device__ inline gs_mf4 gs_mfma(float a, float b, gs_mf4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// acc += block (lane's two complex entries aL = A[l % 8][l / 16], aH = A[l % 8][4 + l / 16]) times
// the right-hand-side values (bL, bH: dofs l / 16 and 4 + l / 16 of column l % 16)
__device__ inline gs_mf4 gs_block_mfma(float2 aL, float2 aH, float2 bL, float2 bH, bool im_row, gs_mf4 acc) {
  acc = gs_mfma(im_row ? aL.y : aL.x, bL.x, acc);
  acc = gs_mfma(im_row ? aH.y : aH.x, bH.x, acc);
  acc = gs_mfma(im_row ? aL.x : -aL.y, bL.y, acc);
  acc = gs_mfma(im_row ? aH.x : -aH.y, bH.y, acc);
  return acc;
}

template <int NB>
__global__ __launch_bounds__(256) void k_stencil_gs_quad_mfma(const float2* __restrict__ A,
                                                                  const float2* __restrict__ Dinv, float2* x,
                                                                  const float2* __restrict__ f, int Lt, int Lx,
                                                                  int qb, int nrhs, int64_t stride,
                                                                  const RhsState* __restrict__ st) {
  static_assert(24 % NB == 0, "batches must cover the 24 offsets");
  constexpr int XS = 9;                   // float2 per (node, rhs) in LDS: 8 dofs + 1 against bank conflicts
  __shared__ float res[4][16][17];        // [node][row][rhs]: f - sum
  __shared__ float nx[4][16][17];         // new values: rows 0..7 Re, 8..15 Im
  __shared__ float2 xs[36 * 16 * XS];     // old values of the group's 6 x 6 neighbourhood
  const int lane = threadIdx.x & 63, v = threadIdx.x >> 6;
  const int rl = lane & 15, kq = lane >> 4, row8 = lane & 7;
  const bool im_row = (lane >> 3) & 1;
  const int qx = Lx >> 2;
  const int grp = blockIdx.x;
  const int t0 = 4 * (grp / qx) + 2 * (qb >> 1), x0 = 4 * (grp % qx) + 2 * (qb & 1);
  const int tn = t0 + (v >> 1), xn = x0 + (v & 1), n = tn * Lx + xn;
  const int rhs = blockIdx.y * 16 + rl;
  const bool live = rhs < nrhs && (!st || st[rhs].active);
  const float2* Ab = A + int64_t(n) * 25 * 64 + row8 * 8 + kq;
  const float2 z2 = make_float2(0.f, 0.f);
  // the neighbourhood rows t0 - 2 .. t0 + 3, columns x0 - 2 .. x0 + 3 of the workgroup's 16 rhs,
  // staged once (each node's 8 dofs as four 16-byte loads) instead of each wave loading its
  // node's 24 neighbours; dead rhs read rhs 0's values and are masked where they are used
  {
    const int r0 = blockIdx.y * 16;
    stage<9, 256, float4>(36 * 16 * 4, [&](int q) {
      const int slot = q / 64, rr = (q / 4) % 16, p = q % 4;
      const int m = wrap1(t0 - 2 + slot / 6, Lt) * Lx + wrap1(x0 - 2 + slot % 6, Lx);
      const int rh = r0 + rr < nrhs ? r0 + rr : 0;
      return reinterpret_cast<const float4*>(x + int64_t(rh) * stride + int64_t(m) * 8)[p];
    }, [&](int q, float4 val) {
      const int slot = q / 64, rr = (q / 4) % 16, p = q % 4;
      float2* d = xs + (slot * 16 + rr) * XS + 2 * p;
      d[0] = make_float2(val.x, val.y);
      d[1] = make_float2(val.z, val.w);
    });
    __syncthreads();
  }
  // phase 1, batches of NB offsets (stencil order without the centre): all loads of a batch are
  // issued before its products.  An earlier node's block gets zero right-hand-side values,
  // which leaves the sums unchanged bit for bit; the batch size does not change them either.
  gs_mf4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int bt = 0; bt < 24 / NB; ++bt) {
    float2 aL[NB], aH[NB], bL[NB], bH[NB];
    bool zero[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int q = NB * bt + j, d = q < 12 ? q : q + 1;
      const int dt = d / 5 - 2, dx = d % 5 - 2;
      const int ga = (v >> 1) + dt, gb = (v & 1) + dx;
      zero[j] = (ga >= 0 && ga <= 1 && gb >= 0 && gb <= 1 && 2 * ga + gb < v) || !live;
      const float2* xv = xs + (((ga + 2) * 6 + (gb + 2)) * 16 + rl) * XS;
      aL[j] = Ab[d * 64];
      aH[j] = Ab[d * 64 + 4];
      bL[j] = xv[kq];
      bH[j] = xv[4 + kq];
    }
    // the mask is applied where the values are used: overwriting a load's destination register
    // in a branch would make every load of the batch wait for the one before it
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int q = NB * bt + j, d = q < 12 ? q : q + 1;
      const float2 cL = zero[j] ? z2 : bL[j], cH = zero[j] ? z2 : bH[j];
      if (d & 1) acc1 = gs_block_mfma(aL[j], aH[j], cL, cH, im_row, acc1);
      else acc0 = gs_block_mfma(aL[j], aH[j], cL, cH, im_row, acc0);
    }
  }
  gs_mf4 tot = acc0 + acc1;
  // the earlier nodes' blocks (stencil offsets 6, 7, 8, 11 are (-1,-1), (-1,0), (-1,+1), (0,-1)),
  // the inverse diagonal block and this lane's f values (rows 4 kq + i)
  constexpr int kEarly[4] = {6, 7, 8, 11};
  float2 eL[4], eH[4];
  int ep[4];
  bool eu[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int d = kEarly[k];
    const int dt = d / 5 - 2, dx = d % 5 - 2;
    const int ga = (v >> 1) + dt, gb = (v & 1) + dx;
    eu[k] = ga >= 0 && ga <= 1 && gb >= 0 && gb <= 1 && 2 * ga + gb < v;
    ep[k] = eu[k] ? 2 * ga + gb : 0;
    eL[k] = eu[k] ? Ab[d * 64] : z2;
    eH[k] = eu[k] ? Ab[d * 64 + 4] : z2;
  }
  const float2* Db = Dinv + int64_t(n) * 64 + row8 * 8 + kq;
  const float2 dL = Db[0], dH = Db[4];
  float fv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float2 q = f && live ? f[int64_t(rhs) * stride + int64_t(n) * 8 + 4 * (kq & 1) + i] : z2;
    fv[i] = kq < 2 ? q.x : q.y;
  }
  // phase 2
  for (int s = 0; s < 4; ++s) {
    __syncthreads();                                   // new values of the nodes before s
    if (v == s) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (!eu[k]) continue;
        const float (*src)[17] = nx[ep[k]];
        const float2 bL = make_float2(src[kq][rl], src[8 + kq][rl]);
        const float2 bH = make_float2(src[4 + kq][rl], src[12 + kq][rl]);
        tot = gs_block_mfma(eL[k], eH[k], bL, bH, im_row, tot);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) res[s][4 * kq + i][rl] = fv[i] - tot[i];
    }
    __syncthreads();
    if (v == s) {
      const float (*src)[17] = res[s];
      const float2 bL = make_float2(src[kq][rl], src[8 + kq][rl]);
      const float2 bH = make_float2(src[4 + kq][rl], src[12 + kq][rl]);
      const gs_mf4 o = gs_block_mfma(dL, dH, bL, bH, im_row, gs_mf4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
      for (int i = 0; i < 4; ++i) nx[s][4 * kq + i][rl] = o[i];
    }
  }
  __syncthreads();
  if (live) {
    float2* xw = x + int64_t(rhs) * stride + int64_t(n) * 8;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int dof = 2 * kq + j;
      xw[dof] = make_float2(nx[v][dof][rl], nx[v][dof + 8][rl]);
    }
  }
}

// y = Ainv v for the coarsest level on FP64 matrix cores: a dense complex product of the
// inverse with the right-hand sides, D[rhs][row] = sum_k v_rhs[k] Ainv[row][k], as real
// v_mfma_f64_16x16x4f64 tiles (lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[4 i + l / 16][l % 16], i < 4).  A workgroup owns 16 right-hand sides x 16 rows; its
// kDenseWaves waves take a slice of k each (a multiple of 4; padding contributes zeros) and the
// slices are added in order through LDS.  The product is latency-bound at these sizes (the
// 512 x 512 inverse is 4 MB): 16 slices keep every wave's loads in one batch in flight and put
// 16 times more waves on the chip than a workgroup per tile with one wave.  The inverse is read
// once per 16 right-hand sides.  A single right-hand side pads its tile, which keeps each
// right-hand side's arithmetic the same in every batch.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
__device__ inline mfma_d4 mfma_f64(double a, double b, mfma_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
constexpr int kDenseWaves = 16;

template <typename Vin, typename Vout>
__global__ __launch_bounds__(64 * kDenseWaves) void k_dense_apply_mfma(const double2* __restrict__ Ainv,
                                                                      const Vin* __restrict__ v, Vout* __restrict__ y,
                                                                      int n, int nrhs, int64_t stride,
                                                                      const RhsState* __restrict__ st) {
  __shared__ double2 red[kDenseWaves][256];
  __shared__ int live[16];                                 // the 16 rhs' flags, for the stores
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, lr = lane & 15, lk = lane >> 4;
  const int row0 = blockIdx.x * 16, r0 = blockIdx.y * 16;
  const int ra = r0 + lr;                                  // right-hand side of this lane's A values
  const bool alive = ra < nrhs && (!st || st[ra].active);
  if (threadIdx.x < 16) live[threadIdx.x] = alive;
  const int rb = row0 + lr;                                // row of this lane's B values
  const bool blive = rb < n;
  const int kq = (((n + 3) / 4 + kDenseWaves - 1) / kDenseWaves) * 4;   // k per wave
  const int k0 = min(n, wv * kq), k1 = min(n, k0 + kq);
  const Vin* va = v + int64_t(alive ? ra : 0) * stride;
  const double2* Ab = Ainv + int64_t(blive ? rb : 0) * n;
  mfma_d4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
  // KB k-steps of operands are loaded (unconditionally, from valid addresses) before their
  // products, so that a wave waits for memory once per KB steps.  Steps past k1 multiply zeros:
  // the accumulators start at +0 and never hold -0, so adding them leaves every bit unchanged.
  constexpr int KB = 8;
  for (int kb = k0; kb < k1; kb += 4 * KB) {
    Vin av[KB];
    double2 bv[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int k = kb + 4 * u + lk;
      av[u] = va[k < k1 ? k : 0];
      bv[u] = Ab[k < k1 ? k : 0];
    }
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const bool kin = kb + 4 * u + lk < k1;
      const double2 a = alive && kin ? cconv<double2>(av[u]) : make_double2(0, 0);
      const double2 b = blive && kin ? bv[u] : make_double2(0, 0);
      re = mfma_f64(a.x, b.x, re);
      re = mfma_f64(-a.y, b.y, re);
      im = mfma_f64(a.x, b.y, im);
      im = mfma_f64(a.y, b.x, im);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) red[wv][i * 64 + lane] = make_double2(re[i], im[i]);
  __syncthreads();
  if (wv >= 4) return;
  const int i = wv;                                        // wave i adds the slices of D's rows 4 i + l / 16
  double2 acc = red[0][i * 64 + lane];
#pragma unroll
  for (int q = 1; q < kDenseWaves; ++q) acc = cadd(acc, red[q][i * 64 + lane]);
  const int r = r0 + 4 * i + lk, row = row0 + lr;
  if (live[4 * i + lk] && row < n) y[r * stride + row] = cconv<Vout>(acc);
}

// Unpreconditioned GMRES from x = 0 on the coarsest level (the paper's coarsest-level solver,
// run there to relative tolerance 0.1), FP64 throughout, one workgroup per right-hand side, so
// that a right-hand side's arithmetic is the same in every batch.  Arnoldi with classical
// Gram-Schmidt applied twice and the FGMRES rotation rule; the cycle stops when
// |g_{j+1}| <= tol ||f||, on breakdown (h_{j+1,j} <= 1e-300 ||f||) or after `steps` steps, and
// x = V R^{-1} g.  Thread t owns rows t and t + 1024 of every vector; the basis is kept in
// `basis` [rhs][steps + 1][n] (each thread reads back only the rows it wrote).  The product
// with the column-major matrix Acm[k][row] is latency-bound on one CU, so it keeps many loads
// in flight: the 1024 threads form S = 1024 / RT segments of k (RT = row threads, a power of
// two >= n up to 1024), each reading coalesced column pieces, and the segment sums of a row
// are added in segment order.  Block sums: butterfly within each wave, then the 16 wave sums
// in order.
constexpr int kCgThreads = 1024, kCgWaves = kCgThreads / 64, kCgRows = 2, kCgMaxSteps = 32;

__device__ inline void cg_wave_part(double2 v, double2 (*part)[kCgWaves], int i, int lane, int wv) {
  v.x = wave_sum(v.x);
  v.y = wave_sum(v.y);
  if (lane == 0) part[i][wv] = v;
}

__device__ inline double2 cg_part_total(const double2* p) {
  double2 s = p[0];
  for (int q = 1; q < kCgWaves; ++q) s = cadd(s, p[q]);
  return s;
}

template <typename Vin, typename Vout>
__global__ __launch_bounds__(kCgThreads) void k_coarsest_gmres(const double2* __restrict__ Acm,
                                                               const Vin* __restrict__ f, Vout* __restrict__ x,
                                                               int n, int64_t stride, const RhsState* __restrict__ st,
                                                               double tol, int steps, double2* __restrict__ basis) {
  extern __shared__ double2 dyn[];                      // xs [n], then segment sums [1024] if n < 1024
  __shared__ double2 part[kCgMaxSteps + 1][kCgWaves];
  __shared__ double2 hp[kCgMaxSteps + 1];               // this pass's projections, then y
  __shared__ double2 hsum[kCgMaxSteps + 2];             // Hessenberg column
  __shared__ double2 R[kCgMaxSteps * (kCgMaxSteps + 1) / 2];
  __shared__ double2 g[kCgMaxSteps + 1], sn[kCgMaxSteps];
  __shared__ double cs[kCgMaxSteps];
  __shared__ double beta_s, hn_s;
  __shared__ int stop_s, k_s;
  const int r = blockIdx.x;
  if (st && !st[r].active) return;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  double2* xs = dyn;
  double2* seg_sum = dyn + n;
  int RT = 64;
  while (RT < n && RT < kCgThreads) RT <<= 1;
  const int S = kCgThreads / RT, rl = t % RT, seg = t / RT;
  const int q0 = int(int64_t(n) * seg / S), q1 = int(int64_t(n) * (seg + 1) / S);
  double2* Vb = basis + int64_t(r) * (steps + 1) * n;
  const Vin* fr = f + int64_t(r) * stride;
  Vout* xr = x + int64_t(r) * stride;
  double2 w[kCgRows];
  // Loads in the loops below are unconditional, from clamped rows, so that no branch separates
  // them; the entries of rows past n are set to zero after each loop and never stored.
  int crow[kCgRows], mrow[kCgRows];
  bool own[kCgRows], mown[kCgRows];
#pragma unroll
  for (int i = 0; i < kCgRows; ++i) {
    own[i] = t + kCgThreads * i < n;
    crow[i] = own[i] ? t + kCgThreads * i : n - 1;
    mown[i] = rl + RT * i < n;
    mrow[i] = mown[i] ? rl + RT * i : n - 1;
  }
  // beta = ||f||
  double2 acc = make_double2(0, 0);
#pragma unroll
  for (int i = 0; i < kCgRows; ++i) {
    const int row = t + kCgThreads * i;
    w[i] = row < n ? cconv<double2>(fr[row]) : make_double2(0, 0);
    acc.x += cabs2(w[i]);
  }
  cg_wave_part(acc, part, 0, lane, wv);
  __syncthreads();
  if (t == 0) {
    beta_s = sqrt(cg_part_total(part[0]).x);
    g[0] = make_double2(beta_s, 0);
  }
  __syncthreads();
  const double beta = beta_s;
  if (beta == 0) {
#pragma unroll
    for (int i = 0; i < kCgRows; ++i) {
      const int row = t + kCgThreads * i;
      if (row < n) xr[row] = cconv<Vout>(make_double2(0, 0));
    }
    return;
  }
  const double ib = 1.0 / beta;
#pragma unroll
  for (int i = 0; i < kCgRows; ++i) {
    const int row = t + kCgThreads * i;
    if (row < n) {
      const double2 v = cscale(w[i], ib);
      Vb[row] = v;
      xs[row] = v;
    }
  }
  int k = 0;
  for (int j = 0; j < steps; ++j) {
    __syncthreads();                                     // xs holds v_j
    // w = A v_j: this thread's segment of k for rows rl (+ 1024 when RT = 1024)
    double2 a[kCgRows];
#pragma unroll
    for (int i = 0; i < kCgRows; ++i) a[i] = make_double2(0, 0);
    // four columns' loads at a time, then their products in column order
    int q = q0;
    for (; q + 4 <= q1; q += 4) {
      double2 cv[4][kCgRows];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < kCgRows; ++i) cv[u][i] = Acm[int64_t(q + u) * n + mrow[i]];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 xq = xs[q + u];
#pragma unroll
        for (int i = 0; i < kCgRows; ++i) a[i] = cfma(cv[u][i], xq, a[i]);
      }
    }
    for (; q < q1; ++q) {
      const double2 xq = xs[q];
#pragma unroll
      for (int i = 0; i < kCgRows; ++i) a[i] = cfma(Acm[int64_t(q) * n + mrow[i]], xq, a[i]);
    }
#pragma unroll
    for (int i = 0; i < kCgRows; ++i)
      if (!mown[i]) a[i] = make_double2(0, 0);
    if (S == 1) {                                        // RT = 1024: rl = t, rows are the owned ones
#pragma unroll
      for (int i = 0; i < kCgRows; ++i) w[i] = a[i];
    } else {                                             // n <= RT <= 512: one row per thread
      seg_sum[seg * RT + rl] = a[0];
      __syncthreads();
      if (t < n) {
        double2 v = seg_sum[t];
        for (int q = 1; q < S; ++q) v = cadd(v, seg_sum[q * RT + t]);
        w[0] = v;
      }
    }
    // classical Gram-Schmidt, applied twice: h = V^H w, w -= V h
    for (int pass = 0; pass < 2; ++pass) {
      for (int l = 0; l <= j; ++l) {
        const double2* vl = Vb + int64_t(l) * n;
        double2 p = make_double2(0, 0);
#pragma unroll
        for (int i = 0; i < kCgRows; ++i) p = cfmac(vl[crow[i]], w[i], p);   // w = 0 past n
        cg_wave_part(p, part, l, lane, wv);
      }
      __syncthreads();
      if (t <= j) {
        const double2 h = cg_part_total(part[t]);
        hp[t] = h;
        hsum[t] = pass == 0 ? h : cadd(hsum[t], h);
      }
      __syncthreads();
      for (int l = 0; l <= j; ++l) {
        const double2* vl = Vb + int64_t(l) * n;
        const double2 h = hp[l];
#pragma unroll
        for (int i = 0; i < kCgRows; ++i) w[i] = cfma(vl[crow[i]], make_double2(-h.x, -h.y), w[i]);
      }
#pragma unroll
      for (int i = 0; i < kCgRows; ++i)
        if (!own[i]) w[i] = make_double2(0, 0);
      __syncthreads();                                   // hp and part are rewritten next
    }
    // h_{j+1,j} = ||w||
    acc = make_double2(0, 0);
#pragma unroll
    for (int i = 0; i < kCgRows; ++i) acc.x += cabs2(w[i]);
    cg_wave_part(acc, part, 0, lane, wv);
    __syncthreads();
    if (t == 0) {
      const double hn = sqrt(cg_part_total(part[0]).x);
      hn_s = hn;
      hsum[j + 1] = make_double2(hn, 0);
      for (int i = 0; i < j; ++i) {                      // earlier rotations
        const double2 a0 = hsum[i], b0 = hsum[i + 1];
        const double2 s0 = sn[i];
        const double c0 = cs[i];
        // (c a + s b, -conj(s) a + c b)
        hsum[i] = cfma(s0, b0, cscale(a0, c0));
        hsum[i + 1] = cfma(make_double2(-s0.x, s0.y), a0, cscale(b0, c0));
      }
      const double2 a0 = hsum[j], b0 = hsum[j + 1];
      double c0;
      double2 s0;
      if (a0.x == 0 && a0.y == 0) {
        c0 = 0;
        s0 = make_double2(1, 0);
      } else {
        const double aa = sqrt(cabs2(a0));
        const double nu = sqrt(cabs2(a0) + cabs2(b0));
        c0 = aa / nu;
        // (a / |a|) conj(b) / nu
        s0 = cscale(cmul(a0, cconj(b0)), 1.0 / (aa * nu));
      }
      cs[j] = c0;
      sn[j] = s0;
      hsum[j] = cfma(s0, b0, cscale(a0, c0));
      for (int i = 0; i <= j; ++i) R[j * (j + 1) / 2 + i] = hsum[i];
      const double2 gj = g[j];
      g[j + 1] = cmul(make_double2(-s0.x, s0.y), gj);
      g[j] = cscale(gj, c0);
      k_s = j + 1;
      stop_s = sqrt(cabs2(g[j + 1])) <= tol * beta || hn <= 1e-300 * beta;
    }
    __syncthreads();
    k = k_s;
    if (stop_s) break;
    const double ih = 1.0 / hn_s;
#pragma unroll
    for (int i = 0; i < kCgRows; ++i) {
      const int row = t + kCgThreads * i;
      if (row < n) {
        const double2 v = cscale(w[i], ih);
        Vb[int64_t(j + 1) * n + row] = v;
        xs[row] = v;
      }
    }
  }
  // y = R^{-1} g (back substitution), x = V y
  if (t == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double2 v = g[i];
      for (int l = i + 1; l < k; ++l) v = cfma(R[l * (l + 1) / 2 + i], make_double2(-hp[l].x, -hp[l].y), v);
      hp[i] = cdiv(v, R[i * (i + 1) / 2 + i]);
    }
  }
  __syncthreads();
  double2 xv[kCgRows];
#pragma unroll
  for (int i = 0; i < kCgRows; ++i) xv[i] = make_double2(0, 0);
  for (int l = 0; l < k; ++l) {
    const double2* vl = Vb + int64_t(l) * n;
    const double2 y = hp[l];
#pragma unroll
    for (int i = 0; i < kCgRows; ++i) xv[i] = cfma(vl[crow[i]], y, xv[i]);
  }
#pragma unroll
  for (int i = 0; i < kCgRows; ++i) {
    const int row = t + kCgThreads * i;
    if (row < n) xr[row] = cconv<Vout>(xv[i]);
  }
}

// Acm[k][row] = A[row][k] (dense n x n)
__global__ void k_transpose_dense(const double2* __restrict__ A, double2* __restrict__ At, int n) {
  __shared__ double2 tile[16][17];
  const int bx = blockIdx.x * 16, by = blockIdx.y * 16;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  if (by + ty < n && bx + tx < n) tile[ty][tx] = A[int64_t(by + ty) * n + bx + tx];
  __syncthreads();
  if (bx + ty < n && by + tx < n) At[int64_t(bx + ty) * n + by + tx] = tile[tx][ty];
}

// ------------------------------------------------------------------------------ launchers

template <int B, typename R, typename M, typename V>
static void apply_b(hipStream_t s, const void* A, const void* x, void* y, const void* f, int Lt,
                    int Lx, int nrhs, int64_t stride, const RhsState* st) {
  const int nn = Lt * Lx;
  dim3 g(unsigned((nn + Lanes<B>::NPB - 1) / Lanes<B>::NPB), unsigned(nrhs));
  hipLaunchKernelGGL((k_stencil_apply<B, R, M, V, V>), g, dim3(256), 0, s, (const M*)A, (const V*)x,
                     (V*)y, (const V*)f, Lt, Lx, stride, st);
}

template <int B, typename R, typename M, typename V>
static void gs_b(hipStream_t s, const void* A, const void* D, void* x, const void* f, int Lt, int Lx,
                 int colour, int nrhs, int64_t stride, const RhsState* st) {
  const int ncn = (Lt / 4) * (Lx / 4);
  dim3 g(unsigned((ncn + Lanes<B>::NPB - 1) / Lanes<B>::NPB), unsigned(nrhs));
  AMAMG_LAUNCH((k_stencil_gs<B, R, M, V>), g, dim3(256), 0, s, (const M*)A, (const M*)D, (V*)x,
                     (const V*)f, Lt, Lx, colour, stride, st);
}

// rb = right-hand sides per wave of the paired sweep for FP32 8 x 8 blocks (1, 2 or 4; 0 = the
// default 2; bitwise the same results for every choice), measured at 32 x 32 nodes, 64 rhs: 11.0
// us per launch with 2 against 14.7 with 1, 11.6 with 4, 19.3 with 8.  FP64 would not fit the
// registers; other block sizes take one right-hand side per wave.
template <int B, typename R, typename M, typename V>
static void gs_pair_b(hipStream_t s, const void* A, const void* D, void* x, const void* f, int Lt, int Lx,
                      int c0, int nrhs, int64_t stride, const RhsState* st, int rb) {
  const int ncn = (Lt / 4) * (Lx / 4);
  if constexpr (B == 8) {
    if (rb == 0 && sizeof(R) == 4) rb = 2;
    if (rb > 1 && nrhs >= rb) {
      const dim3 g(unsigned((ncn + 3) / 4), unsigned((nrhs + rb - 1) / rb));
      if (rb == 4)
        AMAMG_LAUNCH((k_stencil_gs_pair_mr<4, R, M, V>), g, dim3(256), 0, s, (const M*)A, (const M*)D, (V*)x,
                     (const V*)f, Lt, Lx, c0, nrhs, stride, st);
      else
        AMAMG_LAUNCH((k_stencil_gs_pair_mr<2, R, M, V>), g, dim3(256), 0, s, (const M*)A, (const M*)D, (V*)x,
                     (const V*)f, Lt, Lx, c0, nrhs, stride, st);
      return;
    }
  }
  dim3 g(unsigned((ncn + Lanes<B>::NPB - 1) / Lanes<B>::NPB), unsigned(nrhs));
  AMAMG_LAUNCH((k_stencil_gs_pair<B, R, M, V>), g, dim3(256), 0, s, (const M*)A, (const M*)D, (V*)x,
               (const V*)f, Lt, Lx, c0, stride, st);
}

// Colour block qb of the coarse sweep.  FP32 8 x 8 blocks with gs_on_matrix_cores(mode):
// one matrix-core launch, variant = stencil offsets per load batch (8, 12 or 24; 0 = 12).
// Smaller grids, FP64 and other blocks: variant > 0 colour-pair launches with that many
// right-hand sides per wave (8 x 8 blocks; 0 = 2 in FP32, the generic pair kernel in FP64),
// -1 and -2 one k_stencil_gs_quad_mr launch with -variant right-hand sides per wave, and
// kGsNodeWaves one k_stencil_gs_node4 launch (8 x 8 blocks; otherwise colour pairs).  Within each of the two paths every variant gives bitwise the same
// results; which path runs depends on the grid only, so a right-hand side's result does not
// depend on its batch.
template <int B, typename R, typename M, typename V>
static void gs_block_b(hipStream_t s, const void* A, const void* D, void* x, const void* f, int Lt, int Lx,
                       int qb, int nrhs, int64_t stride, const RhsState* st, int variant, int mode) {
  if constexpr (B == 8 && std::is_same<R, float>::value && std::is_same<V, float2>::value &&
                std::is_same<M, float2>::value) {
    if (gs_on_matrix_cores(Lt, Lx, mode)) {
      const int ngr = (Lt / 4) * (Lx / 4);
      const dim3 g(unsigned(ngr), unsigned((nrhs + 15) / 16));
#define AMAMG_GS_MFMA(NB)                                                                      \
  AMAMG_LAUNCH((k_stencil_gs_quad_mfma<NB>), g, dim3(256), 0, s, (const float2*)A, (const float2*)D, \
               (float2*)x, (const float2*)f, Lt, Lx, qb, nrhs, stride, st)
      if (variant == 8) AMAMG_GS_MFMA(8);
      else if (variant == 24) AMAMG_GS_MFMA(24);
      else AMAMG_GS_MFMA(12);
#undef AMAMG_GS_MFMA
      return;
    }
  }
  if constexpr (B == 8) {
    if (variant == kGsNodeWaves) {
      const dim3 g(unsigned((Lt / 4) * (Lx / 4)), unsigned(nrhs));
      AMAMG_LAUNCH((k_stencil_gs_node4<R, M, V>), g, dim3(256), 0, s, (const M*)A, (const M*)D, (V*)x,
                   (const V*)f, Lt, Lx, qb, nrhs, stride, st);
      return;
    }
    const int rb = -variant;
    if ((rb == 1 || rb == 2) && nrhs >= rb) {
      const int ngr = (Lt / 4) * (Lx / 4);
      const dim3 g(unsigned((ngr + 1) / 2), unsigned((nrhs + rb - 1) / rb));
      if (rb == 2)
        AMAMG_LAUNCH((k_stencil_gs_quad_mr<2, R, M, V>), g, dim3(256), 0, s, (const M*)A, (const M*)D, (V*)x,
                     (const V*)f, Lt, Lx, qb, nrhs, stride, st);
      else
        AMAMG_LAUNCH((k_stencil_gs_quad_mr<1, R, M, V>), g, dim3(256), 0, s, (const M*)A, (const M*)D, (V*)x,
                     (const V*)f, Lt, Lx, qb, nrhs, stride, st);
      return;
    }
  }
  const int rb = variant > 0 ? variant : 0;
  gs_pair_b<B, R, M, V>(s, A, D, x, f, Lt, Lx, coarse_colour(4 * qb), nrhs, stride, st, rb);
  gs_pair_b<B, R, M, V>(s, A, D, x, f, Lt, Lx, coarse_colour(4 * qb + 2), nrhs, stride, st, rb);
}

#define AMAMG_B_DISPATCH(fn, prec, ...)                                                       \
  do {                                                                                        \
    if (prec == F64) {                                                                        \
      switch (b) {                                                                            \
        case 2: fn<2, double, double2, double2>(__VA_ARGS__); break;                          \
        case 4: fn<4, double, double2, double2>(__VA_ARGS__); break;                          \
        case 8: fn<8, double, double2, double2>(__VA_ARGS__); break;                          \
        case 16: fn<16, double, double2, double2>(__VA_ARGS__); break;                        \
        case 32: fn<32, double, double2, double2>(__VA_ARGS__); break;                        \
        case 64: fn<64, double, double2, double2>(__VA_ARGS__); break;                        \
        default: break;                                                                       \
      }                                                                                       \
    } else {                                                                                  \
      switch (b) {                                                                            \
        case 2: fn<2, float, float2, float2>(__VA_ARGS__); break;                             \
        case 4: fn<4, float, float2, float2>(__VA_ARGS__); break;                             \
        case 8: fn<8, float, float2, float2>(__VA_ARGS__); break;                             \
        case 16: fn<16, float, float2, float2>(__VA_ARGS__); break;                           \
        case 32: fn<32, float, float2, float2>(__VA_ARGS__); break;                           \
        case 64: fn<64, float, float2, float2>(__VA_ARGS__); break;                           \
        default: break;                                                                       \
      }                                                                                       \
    }                                                                                         \
  } while (0)

void stencil_apply(hipStream_t s, Real prec, const void* A, const void* x, void* y, const void* f,
                   int Lt, int Lx, int b, int nrhs, int64_t stride, const RhsState* st) {
  AMAMG_B_DISPATCH(apply_b, prec, s, A, x, y, f, Lt, Lx, nrhs, stride, st);
}

void stencil_gs(hipStream_t s, Real prec, const void* A, const void* Dinv, void* x, const void* f,
                int Lt, int Lx, int b, int colour, int nrhs, int64_t stride, const RhsState* st) {
  AMAMG_B_DISPATCH(gs_b, prec, s, A, Dinv, x, f, Lt, Lx, colour, nrhs, stride, st);
}


void stencil_gs_block(hipStream_t s, Real prec, const void* A, const void* Dinv, void* x, const void* f,
                      int Lt, int Lx, int b, int qb, int nrhs, int64_t stride, const RhsState* st, int variant,
                      int mode) {
  AMAMG_B_DISPATCH(gs_block_b, prec, s, A, Dinv, x, f, Lt, Lx, qb, nrhs, stride, st, variant, mode);
}

void dense_apply(hipStream_t s, Real prec, const double2* Ainv, const void* v, void* y, int n,
                 int nrhs, int64_t stride, const RhsState* st) {
  // one kernel for every batch size: a right-hand side's result must not depend on the batch
  const dim3 g(unsigned((n + 15) / 16), unsigned((nrhs + 15) / 16));
  if (prec == F64)
    hipLaunchKernelGGL((k_dense_apply_mfma<double2, double2>), g, dim3(64 * kDenseWaves), 0, s, Ainv,
                       (const double2*)v, (double2*)y, n, nrhs, stride, st);
  else
    hipLaunchKernelGGL((k_dense_apply_mfma<float2, float2>), g, dim3(64 * kDenseWaves), 0, s, Ainv,
                       (const float2*)v, (float2*)y, n, nrhs, stride, st);
}

void coarsest_gmres(hipStream_t s, Real prec, const double2* Acm, const void* f, void* x, int n, int nrhs,
                    int64_t stride, const RhsState* st, double tol, int steps, double2* basis) {
  const size_t lds = sizeof(double2) * (size_t(n) + (n < kCgThreads ? kCgThreads : 0));
  if (prec == F64)
    hipLaunchKernelGGL((k_coarsest_gmres<double2, double2>), dim3(unsigned(nrhs)), dim3(kCgThreads), lds, s, Acm,
                       (const double2*)f, (double2*)x, n, stride, st, tol, steps, basis);
  else
    hipLaunchKernelGGL((k_coarsest_gmres<float2, float2>), dim3(unsigned(nrhs)), dim3(kCgThreads), lds, s, Acm,
                       (const float2*)f, (float2*)x, n, stride, st, tol, steps, basis);
}

void transpose_dense(hipStream_t s, const double2* A, double2* At, int n) {
  const dim3 g(unsigned((n + 15) / 16), unsigned((n + 15) / 16));
  hipLaunchKernelGGL(k_transpose_dense, g, dim3(256), 0, s, A, At, n);
}

}  // namespace amamg

