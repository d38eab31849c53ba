// FGMRES(m) kernels, FP64 (paper: FGMRES outer solver, relative tolerance 1e-10).
//
// Right-preconditioned flexible Arnoldi, orthogonalised by classical Gram-Schmidt with a delayed
// second pass (DCGS2: Bielich, Langou, Thomas, Swirydowicz, Yamazaki, Boman, "Low-synch
// Gram-Schmidt with delayed reorthogonalization for Krylov solvers", Parallel Computing 112
// (2022)).  Basis slot j holds u_j, the new direction projected once, until step j finalises it:
//
//   pass A (k_gram):        s = V_<j^H u_j, alpha = ||u_j||^2, t = V_<j^H w, beta = u_j^H w
//                           (w = D z_j, z_j = M u_j), one read of slots 0..j and w;
//   control (k_lag_control): rho_j = sqrt(alpha - ||s||^2); column j-1 of the Hessenberg
//                           matrix gains s and h_{j,j-1} = rho_j, is rotated and tested; then
//                           v_j = (u_j - V_<j s) / rho_j and, for z^_j = z_j / rho_j,
//                           h_<j = t / rho_j, h_j = (beta - s^H t) / rho_j^2;
//   pass B (k_lag_update):  v_j in place of u_j and u_{j+1} = w / rho_j - V_<j h_<j - v_j h_j
//                           into slot j+1, one read of slots 0..j and w.
//
// A cycle of m steps ends with pass A on slots 0..m alone, which finalises column m-1.  In
// exact arithmetic the basis, the Hessenberg matrix and hence the iterates are those of FGMRES
// with classical Gram-Schmidt applied twice; the preconditioner sees u_j instead of v_j, which
// FGMRES allows (its search directions are arbitrary) and which for the linear V-cycle spans
// the same space.  The solution update uses z^_i = z_i / rho_i.  Slot 0 holds v_0 = r / ||r||
// exactly (rho_0 = 1, s empty).
//
// Every reduction is two-level and fixed-order: each block writes its partial sums, and the
// consumer adds them in block order, so results are bitwise reproducible.
//
// Givens rotation for (a, b) = (H_jj, H_{j+1,j}): nu = sqrt(|a|^2 + |b|^2), c = |a| / nu,
// s = (a / |a|) conj(b) / nu (c = 0, s = 1 when a = 0); a rotation maps (x, y) to
// (c x + s y, -conj(s) x + c y); g_{j+1} = -conj(s) g_j, g_j = c g_j.
//
// Vector layouts: basis V [slot][rhs][n], search directions Z [j][rhs][n], w and x [rhs][n].
#include <algorithm>
#include <array>
#include <utility>

#include "launch.hpp"

namespace amamg {

#define KMAXV 32
// partial-sum slot of the Gram pass per block: dots with u at [0, nv), with w at [KMAXV, KMAXV + nv)
#define KGRAM 64

// Basis slots and search directions are streamed: a batch's basis is far larger than the
// caches, so their loads are marked non-temporal and leave L2 and the last-level cache to the
// vectors that are reused.
__device__ inline double2 stream_load(const double2* p) {
  return make_double2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}
__device__ inline float2 stream_load(const float2* p) {
  return make_float2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}
// The finished basis vector v_j is read again only by later steps' passes over the basis.
__device__ inline void stream_store(double2* p, double2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}

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

// fin[i] = sum over blocks of part_r[blk * STRIDE + i] for i < nv, added in a fixed order (8
// strided groups of blocks with eight independent partial sums each, then the groups in order).
// A thread's blocks (at most kSumGroups * 8 of them) are all loaded before the first add, so
// the reduction costs one memory round trip.  Must be called by all 256 threads; fin and
// scratch are shared arrays.
constexpr int kSumGroups = 4;                 // groups of 64 blocks
static_assert(64 * kSumGroups >= kMaxKrylovBlocks, "every block's partial is loaded");
template <int STRIDE>
__device__ inline void sum_blocks(const double2* __restrict__ part_r, int nblk, int nv,
                                  double2* fin, double2* scratch) {
  const int i = threadIdx.x & (KMAXV - 1), c = threadIdx.x / KMAXV;
  double2 s = make_double2(0, 0);
  if (i < nv) {
    double2 pv[kSumGroups][8];
#pragma unroll
    for (int g = 0; g < kSumGroups; ++g)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int b = c + 64 * g + 8 * u;
        pv[g][u] = part_r[int64_t(b < nblk ? b : 0) * STRIDE + i];
      }
    double2 q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) q[u] = make_double2(0, 0);
#pragma unroll
    for (int g = 0; g < kSumGroups; ++g)
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (c + 64 * g + 8 * u < nblk) q[u] = cadd(q[u], pv[g][u]);
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


// Completes Hessenberg column j = a.j of one rhs: col[0..j] holds its projections and
// col[j + 1] = hn = h_{j+1,j}; the earlier rotations csl/snl (all in LDS).  Rotates the
// column, forms rotation j, updates g and tests the end of the cycle; the caller writes the
// column back to H.
__device__ inline void arnoldi_step(const KrylovDims& dm, RhsState& s, int r, double hn, double2* col,
                                    const double* csl, const double2* snl, const ArnoldiArgs& a, double2 gj) {
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

// Lanes per element of the Gram and update passes; lane `sub` holds the slots i = sub + S k.
// Measured cache-cold at 64 rhs x 131072 unknowns: S = 2 is within 2 % of the fastest choice
// from 3 to 20 slots (S = 8 is up to 2x slower); above 24 slots S = 4 bounds the registers.
constexpr int gram_lanes(int nv) { return nv <= 2 ? 1 : nv <= 24 ? 2 : 4; }
constexpr int update_lanes(int nv) { return nv <= 2 ? 1 : nv <= 24 ? 2 : 4; }

// Pass A: partials of V^H u into part[.][0, NV) and (HAS_W) of V^H w into part[.][KMAXV,
// KMAXV + NV), over slots 0..NV-1, where u is slot NV-1 itself.  Each basis value is read
// from memory once; u and w are read once per element and shared by the element's lanes.
// One block's share (block blk of right-hand side r, of dm.nblk per rhs) of pass A.
template <int NV, int S, bool HAS_W>
__device__ inline void gram_item(const KrylovDims& dm, const double2* __restrict__ V, int64_t vsj,
                                 const double2* __restrict__ w, double2* __restrict__ part,
                                 const RhsState* __restrict__ st, int r, int blk) {
  constexpr int K = (NV + S - 1) / S, EPB = 256 / S;
  if (!st[r].active) return;
  __shared__ double2 red[4][KGRAM];
  const int sub = threadIdx.x % S;
  double2 au[K], aw[K];
#pragma unroll
  for (int k = 0; k < K; ++k) au[k] = aw[k] = make_double2(0, 0);
  const double2* Vr = V + r * dm.n;
  const double2* ur = Vr + int64_t(NV - 1) * vsj;
  const double2* wr = HAS_W ? w + r * dm.n : nullptr;
#pragma unroll 1
  for (int64_t d = int64_t(blk) * EPB + threadIdx.x / S; d < dm.n; d += int64_t(dm.nblk) * EPB) {
    // every lane loads, slots past the last clamped to it: their sums are never stored (only
    // slots i < NV are), and a masked load would become a branch that waits for every load in
    // flight.  The scheduling barrier keeps all of the element's loads ahead of the products, so
    // that they are in flight together.
    double2 v[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
      v[k] = stream_load(Vr + (k + 1 < K ? sub + S * k : min(sub + S * k, NV - 1)) * vsj + d);
    const double2 ud = ur[d];
    const double2 wd = HAS_W ? wr[d] : make_double2(0, 0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < K; ++k) au[k] = cfmac(v[k], ud, au[k]);
    if constexpr (HAS_W) {
#pragma unroll
      for (int k = 0; k < K; ++k) aw[k] = cfmac(v[k], wd, aw[k]);
    }
  }
  // block totals: lanes with equal `sub` hold the same slots (xor offsets S .. 32 within a
  // wave), then the four waves in order
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double2 a = au[k], b = aw[k];
#pragma unroll
    for (int o = S; o < 64; o <<= 1) {
      a.x += __shfl_xor(a.x, o);
      a.y += __shfl_xor(a.y, o);
      if constexpr (HAS_W) {
        b.x += __shfl_xor(b.x, o);
        b.y += __shfl_xor(b.y, o);
      }
    }
    const int i = sub + S * k;
    if (lane < S && i < NV) {
      red[wv][i] = a;
      if constexpr (HAS_W) red[wv][KMAXV + i] = b;
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < NV || (HAS_W && t >= KMAXV && t < KMAXV + NV)) {
    double2 a = red[0][t];
    for (int q = 1; q < 4; ++q) a = cadd(a, red[q][t]);
    part[(int64_t(r) * dm.nblk + blk) * KGRAM + t] = a;
  }
  __syncthreads();                                     // red is reused by the next item
}

template <int NV, int S, bool HAS_W>
__global__ __launch_bounds__(256) void k_gram(KrylovDims dm, const double2* __restrict__ V,
                                              int64_t vsj, const double2* __restrict__ w,
                                              double2* __restrict__ part,
                                              const RhsState* __restrict__ st) {
  gram_item<NV, S, HAS_W>(dm, V, vsj, w, part, st, int(blockIdx.y), int(blockIdx.x));
}

// Pass B: v = sum_{i<NV} a_i V_i into slot NV-1 (when write_v; slot 0 is already final) and
// u_next = inv w + sum_{i<NV} b_i V_i into slot NV, with a = coef[r][0, NV), b = coef[r][KMAXV,
// KMAXV + NV) and inv = coef[r][KGRAM - 1].x.  Slot NV-1 is overwritten in place: each element
// is read before it is written, by the same lanes.
template <int NV, int S>
__device__ inline void lag_update_item(const KrylovDims& dm, double2* __restrict__ V, int64_t vsj,
                                       const double2* __restrict__ w, const double2* __restrict__ coef,
                                       const RhsState* __restrict__ st, int write_v, int r, int blk) {
  constexpr int K = (NV + S - 1) / S, EPB = 256 / S;
  if (!st[r].active) return;
  const int sub = threadIdx.x % S;
  const double2* cr = coef + int64_t(r) * KGRAM;
  double2 ak[K], bk[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = sub + S * k;
    ak[k] = i < NV ? cr[i] : make_double2(0, 0);
    bk[k] = i < NV ? cr[KMAXV + i] : make_double2(0, 0);
  }
  const double inv = cr[KGRAM - 1].x;
  double2* Vr = V + r * dm.n;
  const double2* wr = w + r * dm.n;
  double2* vo = Vr + int64_t(NV - 1) * vsj;
  double2* uo = Vr + int64_t(NV) * vsj;
#pragma unroll 1
  for (int64_t d = int64_t(blk) * EPB + threadIdx.x / S; d < dm.n; d += int64_t(dm.nblk) * EPB) {
    double2 v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = sub + S * k;
      v[k] = i < NV ? stream_load(Vr + i * vsj + d) : make_double2(0, 0);
    }
    double2 pa = make_double2(0, 0), pb = make_double2(0, 0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      pa = cfma(v[k], ak[k], pa);
      pb = cfma(v[k], bk[k], pb);
    }
#pragma unroll
    for (int o = 1; o < S; o <<= 1) {
      pa.x += __shfl_xor(pa.x, o);
      pa.y += __shfl_xor(pa.y, o);
      pb.x += __shfl_xor(pb.x, o);
      pb.y += __shfl_xor(pb.y, o);
    }
    if (sub == 0) {
      const double2 wd = wr[d];
      if (write_v) stream_store(vo + d, pa);
      uo[d] = cfma(wd, make_double2(inv, 0.0), pb);
    }
  }
}

template <int NV, int S>
__global__ __launch_bounds__(256) void k_lag_update(KrylovDims dm, double2* __restrict__ V, int64_t vsj,
                                                    const double2* __restrict__ w,
                                                    const double2* __restrict__ coef,
                                                    const RhsState* __restrict__ st, int write_v) {
  lag_update_item<NV, S>(dm, V, vsj, w, coef, st, write_v, int(blockIdx.y), int(blockIdx.x));
}

// Control of step j, one block per rhs, after pass A over slots 0..j (with w when has_w): for
// j > 0 finalises Hessenberg column j-1 (adds s, h_{j,j-1} = rho_j, rotations, convergence);
// then, while the rhs goes on and w was given, writes the pass-B coefficients, column j's
// projections onto slots 0..j and the search-direction scale 1 / rho_j.
__device__ inline void lag_control_item(const KrylovDims& dm, const double2* __restrict__ part,
                                        RhsState* __restrict__ st, const ArnoldiArgs& aa,
                                        double2* __restrict__ coef, double* __restrict__ zsc, int has_w,
                                        int r) {
  __shared__ double2 du[KMAXV], dw[KMAXV], scratch[8 * KMAXV];
  __shared__ double2 col[KMAXV + 1], snl[KMAXV];
  __shared__ double csl[KMAXV];
  __shared__ double rho_sh;
  __shared__ int go;
  const int m = dm.m, j = aa.j, nv = j + 1, t = threadIdx.x;   // j < KMAXV < blockDim.x
  double2* Hr = aa.H + int64_t(r) * (m + 1) * m;
  // the serial section's reads (column j - 1 of H, the rotations, the state and g_{j-1}) are
  // issued before the partial sums' loads, so that they share one memory round trip
  double2 h_old = make_double2(0, 0), sn_old = make_double2(0, 0), g_old = make_double2(0, 0);
  double cs_old = 0.0;
  RhsState s0 = {};
  if (j > 0 && t < j) h_old = Hr[t * m + j - 1];
  if (t + 1 < j) {
    cs_old = aa.cs[int64_t(r) * m + t];
    sn_old = aa.sn[int64_t(r) * m + t];
  }
  if (t == 0) {
    s0 = st[r];
    if (j > 0) g_old = aa.g[int64_t(r) * (m + 1) + j - 1];
  }
  if (!st[r].active) return;                           // uniform over the workgroup
  const double2* pr = part + int64_t(r) * dm.nblk * KGRAM;
  sum_blocks<KGRAM>(pr, dm.nblk, nv, du, scratch);
  if (has_w) sum_blocks<KGRAM>(pr + KMAXV, dm.nblk, nv, dw, scratch);
  if (j > 0) {
    if (t < j) col[t] = cadd(h_old, du[t]);
    if (t + 1 < j) {
      csl[t] = cs_old;
      snl[t] = sn_old;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double ssq = 0.0;
      for (int i = 0; i < j; ++i) ssq += cabs2(du[i]);
      const double rho = sqrt(fmax(du[j].x - ssq, 0.0));
      col[j] = make_double2(rho, 0.0);
      RhsState s = s0;
      ArnoldiArgs a1 = aa;
      a1.j = j - 1;
      arnoldi_step(dm, s, r, rho, col, csl, snl, a1, g_old);
      st[r] = s;
      rho_sh = rho;
      go = s.active && has_w;
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j; i += blockDim.x) Hr[i * m + j - 1] = col[i];
  } else {
    if (threadIdx.x == 0) {
      rho_sh = 1.0;
      go = has_w;
    }
    __syncthreads();
  }
  if (!go || threadIdx.x != 0) return;
  const double inv = 1.0 / rho_sh;
  double2 e = dw[j];                                   // beta - s^H t
  for (int i = 0; i < j; ++i) e = csub(e, cmulc(du[i], dw[i]));
  const double2 ce = cscale(e, inv * inv);             // h_j of z^_j
  double2* cr = coef + int64_t(r) * KGRAM;
  for (int i = 0; i < j; ++i) {
    const double2 ai = cscale(du[i], -inv);
    const double2 ct = cscale(dw[i], inv);
    cr[i] = ai;
    cr[KMAXV + i] = csub(cscale(ct, -1.0), cmul(ce, ai));
    Hr[i * m + j] = ct;
  }
  cr[j] = make_double2(inv, 0.0);
  cr[KMAXV + j] = cscale(ce, -inv);
  cr[KGRAM - 1] = make_double2(inv, 0.0);
  Hr[j * m + j] = ce;
  zsc[int64_t(r) * m + j] = inv;
}

__global__ __launch_bounds__(256) void k_lag_control(KrylovDims dm, const double2* __restrict__ part,
                                                     RhsState* __restrict__ st, ArnoldiArgs aa,
                                                     double2* __restrict__ coef,
                                                     double* __restrict__ zsc, int has_w) {
  lag_control_item(dm, part, st, aa, coef, zsc, has_w, int(blockIdx.x));
}

// ---- several batches (lattices) in one launch --------------------------------------------
// The same work items as the per-batch kernels (block blk of rhs r of batch q), walked by a
// fixed grid of workgroups: item i goes to workgroup i mod gridDim.x, in increasing order.  An
// item computes exactly what the per-batch kernel's block computes, so every right-hand side
// gets bitwise its result in its own batch.  Items never wait on each other.
__device__ inline int seg_of(const KrylovSeg* __restrict__ seg, int nseg, int item) {
  int q = 0;
  while (q + 1 < nseg && seg[q + 1].item0 <= item) ++q;
  return q;
}

template <int NV, int S, bool HAS_W>
__global__ __launch_bounds__(256) void k_gram_multi(const KrylovSeg* __restrict__ seg, int nseg, int total) {
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const KrylovSeg& q = seg[seg_of(seg, nseg, item)];
    const int i = item - q.item0, r = i / q.dm.nblk, blk = i - r * q.dm.nblk;
    gram_item<NV, S, HAS_W>(q.dm, q.V, q.vsj, HAS_W ? q.w : nullptr, q.part, q.st, r, blk);
  }
}

template <int NV, int S>
__global__ __launch_bounds__(256) void k_lag_update_multi(const KrylovSeg* __restrict__ seg, int nseg, int total,
                                                          int write_v) {
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const KrylovSeg& q = seg[seg_of(seg, nseg, item)];
    const int i = item - q.item0, r = i / q.dm.nblk, blk = i - r * q.dm.nblk;
    lag_update_item<NV, S>(q.dm, q.V, q.vsj, q.w, q.coef, q.st, write_v, r, blk);
  }
}

__global__ __launch_bounds__(256) void k_lag_control_multi(const KrylovSeg* __restrict__ seg, int nseg,
                                                           int total, int j, int has_w) {
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    // rhs items: item0 counts blocks, so the rhs index comes from the prefix of rhs counts
    int qi = 0;
    while (qi + 1 < nseg && seg[qi + 1].rhs0 <= item) ++qi;
    const KrylovSeg& q = seg[qi];
    ArnoldiArgs aa = q.aa;
    aa.j = j;
    __syncthreads();                                   // the previous item's LDS is free
    lag_control_item(q.dm, q.part, q.st, aa, q.coef, q.zsc, has_w, item - q.rhs0);
  }
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
  sum_blocks<KMAXV>(part + int64_t(r) * dm.nblk * KMAXV, dm.nblk, 1, nr, scratch);
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

// y = R^{-1} g (k x k upper triangle of the rotated Hessenberg matrix), then y_i / rho_i for
// the stored directions z_i = rho_i z^_i; marks the rhs for the x update and the true residual
// (active = in_cycle).
__global__ void k_backsolve(KrylovDims dm, RhsState* __restrict__ st, const double2* __restrict__ H,
                            const double2* __restrict__ g, const double* __restrict__ zsc,
                            double2* __restrict__ y) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= dm.nrhs) return;
  RhsState s = st[r];
  const int m = dm.m;
  if (!s.in_cycle || s.k == 0 || s.nonfinite) { s.active = s.in_cycle && !s.nonfinite; st[r] = s; return; }
  const double2* Hr = H + int64_t(r) * (m + 1) * m;
  const double2* gr = g + int64_t(r) * (m + 1);
  const double* zr = zsc + int64_t(r) * m;
  double2* yr = y + int64_t(r) * m;
  for (int i = s.k - 1; i >= 0; --i) {
    double2 acc = gr[i];
    for (int q = i + 1; q < s.k; ++q) acc = csub(acc, cmul(Hr[i * m + q], yr[q]));
    const double2 d = Hr[i * m + i];
    const double den = cabs2(d);
    yr[i] = cmul(acc, make_double2(d.x / den, -d.y / den));
  }
  for (int i = 0; i < s.k; ++i) yr[i] = cscale(yr[i], zr[i]);
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
  const Vz* zr = Z + r * dm.n + d;
  // four search directions' loads in flight at a time; the sum keeps its order
  int i = 0;
  for (; i + 4 <= s.k; i += 4) {
    Vz zv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) zv[u] = stream_load(zr + (i + u) * zsj);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = cfma(cconv<double2>(zv[u]), yr[i + u], acc);
  }
  for (; i < s.k; ++i) acc = cfma(cconv<double2>(stream_load(zr + i * zsj)), yr[i], acc);
  x[r * dm.n + d] = acc;
}

// ------------------------------------------------------------------------------ launchers

template <int NV, bool HAS_W>
void launch_gram(hipStream_t s, const KrylovDims& d, const double2* V, int64_t vsj, const double2* w,
                 double2* part, const RhsState* st) {
  AMAMG_LAUNCH((k_gram<NV, gram_lanes(NV), HAS_W>), dim3(d.nblk, d.nrhs), dim3(256), 0, s, d, V, vsj,
               w, part, st);
}
template <int NV>
void launch_lag_update(hipStream_t s, const KrylovDims& d, double2* V, int64_t vsj, const double2* w,
                       const double2* coef, const RhsState* st, int write_v) {
  AMAMG_LAUNCH((k_lag_update<NV, update_lanes(NV)>), dim3(d.nblk, d.nrhs), dim3(256), 0, s, d, V, vsj,
               w, coef, st, write_v);
}
using GramFn = void (*)(hipStream_t, const KrylovDims&, const double2*, int64_t, const double2*,
                        double2*, const RhsState*);
using LagFn = void (*)(hipStream_t, const KrylovDims&, double2*, int64_t, const double2*,
                       const double2*, const RhsState*, int);
template <bool HAS_W, int... I>
static constexpr std::array<GramFn, sizeof...(I)> table_gram(std::integer_sequence<int, I...>) {
  return {&launch_gram<I + 1, HAS_W>...};
}
template <int... I>
static constexpr std::array<LagFn, sizeof...(I)> table_lag(std::integer_sequence<int, I...>) {
  return {&launch_lag_update<I + 1>...};
}
static const auto kGramW = table_gram<true>(std::make_integer_sequence<int, KMAXV - 1>{});
static const auto kGram = table_gram<false>(std::make_integer_sequence<int, KMAXV>{});
static const auto kLag = table_lag(std::make_integer_sequence<int, KMAXV - 1>{});

// nv (slots 0..nv-1) is at most KMAXV - 1 with w and KMAXV without; the restart length is
// limited to KMAXV - 1 where solves are configured.
void gram(hipStream_t s, const KrylovDims& d, const double2* V, int64_t vsj, int nv, const double2* w,
          double2* part, const RhsState* st) {
  if (w) kGramW[nv - 1](s, d, V, vsj, w, part, st);
  else kGram[nv - 1](s, d, V, vsj, nullptr, part, st);
}

void lag_control(hipStream_t s, const KrylovDims& d, const double2* part, RhsState* st, double2* H,
                 double* cs, double2* sn, double2* g, double2* coef, double* zsc, int j, int has_w,
                 double tol, double inner_tol, int max_iters, double2* hist, int hist_cap) {
  ArnoldiArgs aa{H, cs, sn, g, j, tol, inner_tol, max_iters, hist, hist_cap};
  hipLaunchKernelGGL(k_lag_control, dim3(d.nrhs), dim3(256), 0, s, d, part, st, aa, coef, zsc, has_w);
}

void lag_update(hipStream_t s, const KrylovDims& d, double2* V, int64_t vsj, int nv, const double2* w,
                const double2* coef, const RhsState* st, int write_v) {
  kLag[nv - 1](s, d, V, vsj, w, coef, st, write_v);
}

// several batches: persistent grids of at most kMultiGrid workgroups
constexpr int kMultiGrid = 2048;
static dim3 multi_grid(int items) { return dim3(unsigned(std::max(1, std::min(items, kMultiGrid)))); }

template <int NV, bool HAS_W>
void launch_gram_multi(hipStream_t s, const KrylovSeg* seg, int nseg, int total) {
  AMAMG_LAUNCH((k_gram_multi<NV, gram_lanes(NV), HAS_W>), multi_grid(total), dim3(256), 0, s, seg, nseg, total);
}
template <int NV>
void launch_lag_update_multi(hipStream_t s, const KrylovSeg* seg, int nseg, int total, int write_v) {
  AMAMG_LAUNCH((k_lag_update_multi<NV, update_lanes(NV)>), multi_grid(total), dim3(256), 0, s, seg, nseg, total,
               write_v);
}
using GramMultiFn = void (*)(hipStream_t, const KrylovSeg*, int, int);
using LagMultiFn = void (*)(hipStream_t, const KrylovSeg*, int, int, int);
template <bool HAS_W, int... I>
static constexpr std::array<GramMultiFn, sizeof...(I)> table_gram_multi(std::integer_sequence<int, I...>) {
  return {&launch_gram_multi<I + 1, HAS_W>...};
}
template <int... I>
static constexpr std::array<LagMultiFn, sizeof...(I)> table_lag_multi(std::integer_sequence<int, I...>) {
  return {&launch_lag_update_multi<I + 1>...};
}
static const auto kGramMultiW = table_gram_multi<true>(std::make_integer_sequence<int, KMAXV - 1>{});
static const auto kLagMulti = table_lag_multi(std::make_integer_sequence<int, KMAXV - 1>{});

void gram_multi(hipStream_t s, const KrylovSeg* seg, int nseg, int total_blocks, int nv) {
  kGramMultiW[nv - 1](s, seg, nseg, total_blocks);
}

void lag_control_multi(hipStream_t s, const KrylovSeg* seg, int nseg, int total_rhs, int j, int has_w) {
  hipLaunchKernelGGL(k_lag_control_multi, multi_grid(total_rhs), dim3(256), 0, s, seg, nseg, total_rhs, j, has_w);
}

void lag_update_multi(hipStream_t s, const KrylovSeg* seg, int nseg, int total_blocks, int nv, int write_v) {
  kLagMulti[nv - 1](s, seg, nseg, total_blocks, write_v);
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
                      const double2* g, const double* zsc, double2* y, Real zprec, const void* Z,
                      int64_t zsj, double2* x) {
  hipLaunchKernelGGL(k_backsolve, dim3((d.nrhs + 63) / 64), dim3(64), 0, s, d, st, H, g, zsc, y);
  dim3 grid(unsigned((d.n + 255) / 256), d.nrhs);
  if (zprec == F64)
    hipLaunchKernelGGL((k_update_x<double2>), grid, dim3(256), 0, s, d, st, y, (const double2*)Z, zsj, x);
  else
    hipLaunchKernelGGL((k_update_x<float2>), grid, dim3(256), 0, s, d, st, y, (const float2*)Z, zsj, x);
}

}  // namespace amamg
