// Setup kernels (paper, Multilevel approach section: coarsening, interpolation, Galerkin
// coarse operator; SM-AMG for LQCD subsection: per-wirebasket block system and the
// Schur-complement interpolation).
//
// For each wirebasket W the level operator restricted to W's points is split into F (edge
// and interior) and V (vertex) blocks; P_F^W = -A_FF^{-1} A_FV solves the first two block
// rows of the ideal-presmoothing system and equals both Schur-complement formulas of the
// paper.  Systems are solved by a batched LU with partial pivoting, one workgroup per system.
//
// Local numbering inside a wirebasket: footprint position pos = dt*(a+o) + dx.  The host
// passes postab[pos] = F index (>= 0) or -(1 + vcol) with vcol = c*bc + (pt*o + px)*b the
// first interpolation column of a vertex (corner c = 2*ct + cx), and fpos[fi] = pos of the
// fi-th F position.
#include <type_traits>
#include <utility>

#include "launch.hpp"

namespace amamg {

__device__ inline int wrap_s(int v, int L) { v %= L; return v < 0 ? v + L : v; }

// Aug [W][nfd][nfd + ncol] = [A_FF | -A_FV]; A: block stencil [node][noff][b][b]
__global__ __launch_bounds__(256) void k_gather_local(Geom g, const double2* __restrict__ A, int noff,
                                                      const int* __restrict__ offs,
                                                      const int* __restrict__ postab,
                                                      const int* __restrict__ fpos, int nf,
                                                      double2* __restrict__ Aug) {
  const int w = blockIdx.x;
  const int I = w / g.nJ, J = w - (w / g.nJ) * g.nJ;
  const int fpw = g.a + g.o;
  const int nfd = nf * g.b, ncol = g.nvcol(), ld = nfd + ncol;
  double2* Aw = Aug + int64_t(w) * nfd * ld;
  for (int64_t e = threadIdx.x; e < int64_t(nfd) * ld; e += blockDim.x) Aw[e] = make_double2(0, 0);
  __syncthreads();
  for (int rrow = threadIdx.x; rrow < nfd; rrow += blockDim.x) {
    const int fi = rrow / g.b, i = rrow - (rrow / g.b) * g.b;
    const int pos = fpos[fi];
    const int dt = pos / fpw, dx = pos - (pos / fpw) * fpw;
    const int pt_ = wrap_s(g.a * I + dt, g.Lt), px_ = wrap_s(g.a * J + dx, g.Lx);
    const int p = pt_ * g.Lx + px_;
    for (int d = 0; d < noff; ++d) {
      const int qt = wrap_s(pt_ + offs[2 * d], g.Lt), qx = wrap_s(px_ + offs[2 * d + 1], g.Lx);
      const int ldt = wrap_s(qt - g.a * I, g.Lt), ldx = wrap_s(qx - g.a * J, g.Lx);
      if (ldt >= fpw || ldx >= fpw) continue;
      const int code = postab[ldt * fpw + ldx];
      const double2* blk = A + (int64_t(p) * noff + d) * g.b * g.b + int64_t(i) * g.b;
      if (code >= 0) {
        double2* dst = Aw + int64_t(rrow) * ld + int64_t(code) * g.b;
        for (int j = 0; j < g.b; ++j) dst[j] = cadd(dst[j], blk[j]);
      } else {
        double2* dst = Aw + int64_t(rrow) * ld + nfd + (-code - 1);
        for (int j = 0; j < g.b; ++j) dst[j] = csub(dst[j], blk[j]);
      }
    }
  }
}

// Batched dense solve X = A^{-1} B on the augmented row-major matrix [A | B] (n rows, ld = n +
// nrhs columns).  Blocked right-looking LU with partial pivoting (largest |a_ik|, lowest row
// index on ties; the interchanges are applied to the rows of the current and trailing columns,
// so B is permuted and eliminated along the way), panel width LU_NB; the trailing rank-LU_NB
// updates run on 64 x 64 tiles staged in LDS.  Then a blocked back substitution U X = B' with
// the same tiled update.  On exit the B columns hold X (and the other columns U and the L
// factors, the latter without the later interchanges).  info[sys] = 0, or k + 1 when the
// pivot column k is zero or not finite.
#define LU_NB 16
static_assert(kDenseSolveInts == 1 + LU_NB, "dense_solve: info and the panel interchanges");

// M[r][c] -= sum_{q < kb} M[r][lc + q] * M[ur + q][c]  for r in [r0, r1), c in [c0, c1)
// One 64 x 64 tile of M[r][c] -= sum_{q < kb} M[r][lc + q] * M[ur + q][c], rows [tr, min(tr + 64,
// r1)), columns [tc, min(tc + 64, c1)); all 256 threads, staged in LDS.
__device__ void tile_one(double2* __restrict__ M, int ld, int tr, int tc, int r1, int c1, int lc,
                         int ur, int kb, double2 (*Ls)[LU_NB + 1], double2 (*Us)[64 + 1]) {
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  for (int e = tid; e < 64 * LU_NB; e += 256) {
    const int rr = e / LU_NB, q = e - (e / LU_NB) * LU_NB;
    Ls[rr][q] = (tr + rr < r1 && q < kb) ? M[int64_t(tr + rr) * ld + lc + q] : make_double2(0, 0);
  }
  for (int e = tid; e < LU_NB * 64; e += 256) {
    const int q = e >> 6, cc = e & 63;
    Us[q][cc] = (q < kb && tc + cc < c1) ? M[int64_t(ur + q) * ld + tc + cc] : make_double2(0, 0);
  }
  __syncthreads();
  double2 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0, 0);
  for (int q = 0; q < kb; ++q) {
    double2 lv[4], uv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) lv[a] = Ls[ty * 4 + a][q];
#pragma unroll
    for (int b = 0; b < 4; ++b) uv[b] = Us[q][tx + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = cfma(lv[a], uv[b], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int r = tr + ty * 4 + a;
    if (r >= r1) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int c = tc + tx + 16 * b;
      if (c < c1) M[int64_t(r) * ld + c] = csub(M[int64_t(r) * ld + c], acc[a][b]);
    }
  }
  __syncthreads();
}

// M[r][c] -= sum_{q < kb} M[r][lc + q] * M[ur + q][c]  for r in [r0, r1), c in [c0, c1)
__device__ void tile_update(double2* __restrict__ M, int ld, int r0, int r1, int c0, int c1,
                            int lc, int ur, int kb, double2 (*Ls)[LU_NB + 1],
                            double2 (*Us)[64 + 1]) {
  for (int tr = r0; tr < r1; tr += 64)
    for (int tc = c0; tc < c1; tc += 64) tile_one(M, ld, tr, tc, r1, c1, lc, ur, kb, Ls, Us);
}

// Panel k0 of the LU with partial pivoting (one workgroup per system): pivot search (largest
// |a|^2, lowest index on ties), full-row swap, column scaling and the in-panel update, then
// U12 = L11^{-1} A12 for every column right of the panel.  Returns false on a zero or
// non-finite pivot (info set).
__device__ bool lu_panel(double2* __restrict__ M, int n, int ld, int k0, int sys, int* __restrict__ info,
                         double* sv, int* si) {
  const int tid = threadIdx.x;
  const int kb = min(LU_NB, n - k0);
  for (int k = k0; k < k0 + kb; ++k) {
    double best = -1.0;
    int bi = n;
    for (int i = k + tid; i < n; i += 256) {
      const double v = cabs2(M[int64_t(i) * ld + k]);
      if (v > best) { best = v; bi = i; }
    }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (tid < off) {
        const double v2 = sv[tid + off];
        const int i2 = si[tid + off];
        if (v2 > sv[tid] || (v2 == sv[tid] && i2 < si[tid])) { sv[tid] = v2; si[tid] = i2; }
      }
      __syncthreads();
    }
    const int p = si[0];
    const double pmax = sv[0];
    __syncthreads();
    if (!(pmax > 0.0) || !(pmax < 1e300) || p >= n) {
      if (tid == 0) info[sys] = k + 1;
      return false;
    }
    if (p != k) {
      for (int j = tid; j < ld; j += 256) {
        const double2 t = M[int64_t(k) * ld + j];
        M[int64_t(k) * ld + j] = M[int64_t(p) * ld + j];
        M[int64_t(p) * ld + j] = t;
      }
      __syncthreads();
    }
    const double2 akk = M[int64_t(k) * ld + k];
    const double den = cabs2(akk);
    const double2 inv = make_double2(akk.x / den, -akk.y / den);
    for (int i = k + 1 + tid; i < n; i += 256) {
      double2* Mi = M + int64_t(i) * ld;
      const double2 l = cmul(Mi[k], inv);
      Mi[k] = l;
      for (int j = k + 1; j < k0 + kb; ++j) Mi[j] = csub(Mi[j], cmul(l, M[int64_t(k) * ld + j]));
    }
    __syncthreads();
  }
  // U12 = L11^{-1} A12 for the columns right of the panel (unit lower triangle)
  for (int c = k0 + kb + tid; c < ld; c += 256) {
    for (int r = 1; r < kb; ++r) {
      double2 acc = M[int64_t(k0 + r) * ld + c];
      for (int q = 0; q < r; ++q) acc = csub(acc, cmul(M[int64_t(k0 + r) * ld + k0 + q], M[int64_t(k0 + q) * ld + c]));
      M[int64_t(k0 + r) * ld + c] = acc;
    }
  }
  __syncthreads();
  return true;
}

// Shared memory of the register panel: per-wave pivot candidates (value, row, row values),
// the old row k, the row interchanges and the panel's unit lower triangle, double-buffered
// by step parity so that one barrier per pivot step suffices.
struct PanelSmem {
  double sv[2][4];
  int si[2][4];
  double2 crow[2][4][LU_NB];
  double2 krow[2][LU_NB];
  double2 L11[LU_NB][LU_NB + 1];
  int perm[LU_NB];
};

// c ? a : b, component-wise (a select of values, never of their addresses)
__device__ __forceinline__ double2 sel2(bool c, double2 a, double2 b) {
  return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}

// f(integral_constant<int, K>) for K = 0, 1, ... in order, while it returns true (compile-time
// indices, so that register arrays indexed by K stay in registers)
template <typename F, int... K>
__device__ __forceinline__ bool static_while(F&& f, std::integer_sequence<int, K...>) {
  return (f(std::integral_constant<int, K>{}) && ...);
}

// Panel k0 (width NB <= LU_NB) as lu_panel factors it (the same pivots and operations in order),
// with the panel's rows k0 .. n - 1 in registers: thread t holds rows k0 + t + 256 s, s < S
// (n - k0 <= 256 S, 256 threads).  A pivot step is one wave reduction and one barrier.  The
// factored panel columns are written back; the interchanges (sm.perm) and the panel's unit
// lower triangle (sm.L11) are left for lu_columns, which applies them to the columns right of
// the panel.  Columns left of the panel (earlier L factors, which the solve never reads again)
// are not interchanged.
template <int S, int NB = LU_NB>
__device__ __forceinline__ bool lu_panel_reg(double2* __restrict__ M, int n, int ld, int k0, int sys,
                                             int* __restrict__ info, PanelSmem& sm) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int kb = min(NB, n - k0), m = n - k0;
  using Seq = std::make_integer_sequence<int, NB>;
  double2 P[S][NB];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int lr = tid + 256 * s;
    const double2* src = M + int64_t(k0 + (lr < m ? lr : 0)) * ld + k0;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const double2 v = src[q < kb ? q : 0];
      const bool in = lr < m && q < kb;
      P[s][q] = make_double2(in ? v.x : 0.0, in ? v.y : 0.0);
    }
  }
  bool fail = false;   // (set by every thread alike: all read the same pivot from LDS)
  static_while([&](auto kc) __attribute__((always_inline)) -> bool {
    constexpr int k = decltype(kc)::value;
    if (k >= kb) return false;   // (uniform) past the panel: done
    constexpr int par = k & 1;
    double best = -1.0;
    int bi = n;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int lr = tid + 256 * s;
      const double v = cabs2(P[s][k]);
      if (lr >= k && lr < m && v > best) {
        best = v;
        bi = k0 + lr;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double v2 = __shfl_xor(best, off);
      const int i2 = __shfl_xor(bi, off);
      if (v2 > best || (v2 == best && i2 < bi)) {
        best = v2;
        bi = i2;
      }
    }
    if (lane == 0) {
      sm.sv[par][wv] = best;
      sm.si[par][wv] = bi;
    }
    if (bi < n && tid == ((bi - k0) & 255)) {
      const int so = (bi - k0) >> 8;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        double2 v = P[0][q];
#pragma unroll
        for (int s = 1; s < S; ++s) v = sel2(s == so, P[s][q], v);
        sm.crow[par][wv][q] = v;
      }
    }
    if (tid == k)
#pragma unroll
      for (int q = 0; q < NB; ++q) sm.krow[par][q] = P[0][q];
    __syncthreads();
    double pmax = sm.sv[par][0];
    int p = sm.si[par][0], pw = 0;
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      const double v2 = sm.sv[par][w];
      const int i2 = sm.si[par][w];
      if (v2 > pmax || (v2 == pmax && i2 < p)) {
        pmax = v2;
        p = i2;
        pw = w;
      }
    }
    if (!(pmax > 0.0) || !(pmax < 1e300) || p >= n) {
      if (tid == 0) info[sys] = k0 + k + 1;
      fail = true;
      return false;
    }
    if (tid == 0) sm.perm[k] = p;
    double2 prow[NB];
#pragma unroll
    for (int q = k; q < NB; ++q) prow[q] = sm.crow[par][pw][q];
    const int lp = p - k0;
    if (lp != k) {
      if (tid == (lp & 255)) {
        const int so = lp >> 8;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          const double2 v = sm.krow[par][q];
#pragma unroll
          for (int s = 0; s < S; ++s) P[s][q] = sel2(s == so, v, P[s][q]);
        }
      }
      if (tid == k)
#pragma unroll
        for (int q = 0; q < NB; ++q) P[0][q] = sm.crow[par][pw][q];
    }
    const double2 akk = prow[k];
    const double den = cabs2(akk);
    const double2 inv = make_double2(akk.x / den, -akk.y / den);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int lr = tid + 256 * s;
      if (lr > k && lr < m) {
        const double2 l = cmul(P[s][k], inv);
        P[s][k] = l;
#pragma unroll
        for (int j = k + 1; j < NB; ++j)
          if (j < kb) P[s][j] = csub(P[s][j], cmul(l, prow[j]));
      }
    }
    return true;
  }, Seq{});
  if (fail) return false;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int lr = tid + 256 * s;
    if (lr < m)
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (q < kb) M[int64_t(k0 + lr) * ld + k0 + q] = P[s][q];
  }
  if (tid < kb)
#pragma unroll
    for (int q = 0; q < NB; ++q) sm.L11[tid][q] = P[0][q];
  __syncthreads();
  return true;
}

// The columns c0, c0 + cstride, ... counted from the end of panel k0 (B included): the panel's
// row interchanges perm[k] (k < kb, in order) and U12 = L11^{-1} A12 (unit lower triangle),
// one column per thread with the column's panel rows in registers.  Rows that an interchange
// sends out of the panel are tracked in registers too, so each value is loaded and stored once.
__device__ __forceinline__ void lu_columns(double2* __restrict__ M, int ld, int k0, int kb, const int* perm,
                                           const double2 (*L11)[LU_NB + 1], int c0, int cstride) {
  int pm[LU_NB];
#pragma unroll
  for (int k = 0; k < LU_NB; ++k) pm[k] = k < kb ? perm[k] : k0;   // (unused past kb; a valid row)
  const int pe = k0 + kb;   // first row (and column) past the panel
  for (int c = pe + c0; c < ld; c += cstride) {
    // (a compiler barrier: L11 is re-read from LDS per column rather than held in registers)
    __asm__ volatile("" ::: "memory");
    double2 r[LU_NB], e[LU_NB];
#pragma unroll
    for (int q = 0; q < LU_NB; ++q) r[q] = M[int64_t(k0 + (q < kb ? q : 0)) * ld + c];
#pragma unroll
    for (int k = 0; k < LU_NB; ++k) e[k] = M[int64_t(pm[k] >= pe ? pm[k] : k0) * ld + c];
    // the interchanges in order; e[k] = what row pm[k] holds after step k
#pragma unroll
    for (int k = 0; k < LU_NB; ++k) {
      const int pk = pm[k];
      if (k >= kb) {
      } else if (pk < pe) {
#pragma unroll
        for (int q = k + 1; q < LU_NB; ++q)
          if (pk - k0 == q) {
            const double2 t = r[q];
            r[q] = r[k];
            r[k] = t;
          }
      } else {
        double2 cur = e[k];
#pragma unroll
        for (int k2 = 0; k2 < k; ++k2)
          if (pm[k2] == pk) cur = e[k2];
        e[k] = r[k];
        r[k] = cur;
      }
    }
#pragma unroll
    for (int k = 0; k < LU_NB; ++k) {
      bool last = k < kb && pm[k] >= pe;
#pragma unroll
      for (int k2 = k + 1; k2 < LU_NB; ++k2)
        if (k2 < kb && pm[k2] == pm[k]) last = false;
      if (last) M[int64_t(pm[k]) * ld + c] = e[k];
    }
    // U12 = L11^{-1} A12 (unit lower triangle)
#pragma unroll
    for (int rr = 1; rr < LU_NB; ++rr) {
      double2 acc = r[rr];
#pragma unroll
      for (int q = 0; q < rr; ++q) acc = csub(acc, cmul(L11[rr][q], r[q]));
      if (rr < kb) r[rr] = acc;
    }
#pragma unroll
    for (int q = 0; q < LU_NB; ++q)
      if (q < kb) M[int64_t(k0 + q) * ld + c] = r[q];
  }
}

// Diagonal block k0 of the back substitution U X = B' on the right-hand-side columns [n, ld):
// X rows k0 .. k0 + kb for the columns c0 + tid, c0 + tid + stride, ...
__device__ __forceinline__ void back_diag(double2* __restrict__ M, int n, int ld, int k0, int c0, int cstride,
                          double2 (*Ud)[LU_NB + 1]) {
  const int kb = min(LU_NB, n - k0);
  {
    // the diagonal block of U in LDS (LU_NB^2 = 256 entries, one per thread)
    const int r = threadIdx.x / LU_NB, q = threadIdx.x % LU_NB;
    const bool in = r < kb && q < kb;
    const double2 v = M[int64_t(k0 + (in ? r : 0)) * ld + k0 + (in ? q : 0)];
    Ud[r][q] = sel2(in, v, make_double2(0, 0));
  }
  __syncthreads();
  for (int c = n + c0 + threadIdx.x; c < ld; c += cstride) {
    __asm__ volatile("" ::: "memory");   // (Ud re-read from LDS per column, not held in registers)
    double2 x[LU_NB];
#pragma unroll
    for (int q = 0; q < LU_NB; ++q) x[q] = M[int64_t(k0 + (q < kb ? q : 0)) * ld + c];
#pragma unroll
    for (int r = LU_NB - 1; r >= 0; --r) {
      double2 acc = x[r];
#pragma unroll
      for (int q = r + 1; q < LU_NB; ++q)
        if (q < kb) acc = csub(acc, cmul(Ud[r][q], x[q]));
      const double2 d = Ud[r][r];
      const double den = cabs2(d);
      if (r < kb) x[r] = cmul(acc, make_double2(d.x / den, -d.y / den));
    }
#pragma unroll
    for (int q = 0; q < LU_NB; ++q)
      if (q < kb) M[int64_t(k0 + q) * ld + c] = x[q];
  }
  __syncthreads();
}

// n <= 256: the panels in registers.
__global__ __launch_bounds__(256) void k_dense_solve(double2* __restrict__ A, int n, int ld,
                                                     int* __restrict__ info) {
  const int sys = blockIdx.x;
  double2* M = A + int64_t(sys) * n * ld;
  __shared__ PanelSmem psm;
  __shared__ double2 Ls[64][LU_NB + 1];
  __shared__ double2 Us[LU_NB][64 + 1];
  if (threadIdx.x == 0) info[sys] = 0;
  for (int k0 = 0; k0 < n; k0 += LU_NB) {
    if (!lu_panel_reg<1>(M, n, ld, k0, sys, info, psm)) return;
    const int kb = min(LU_NB, n - k0);
    lu_columns(M, ld, k0, kb, psm.perm, psm.L11, threadIdx.x, 256);
    __syncthreads();
    tile_update(M, ld, k0 + kb, n, k0 + kb, ld, k0, k0, kb, Ls, Us);
    __syncthreads();
  }
  // back substitution U X = B' on the right-hand-side columns
  const int last = ((n - 1) / LU_NB) * LU_NB;
  for (int k0 = last; k0 >= 0; k0 -= LU_NB) {
    const int kb = min(LU_NB, n - k0);
    back_diag(M, n, ld, k0, 0, 256, psm.L11);
    if (k0 > 0) tile_update(M, ld, 0, k0, n, ld, k0, k0, kb, Ls, Us);
    __syncthreads();
  }
}

// The same factorisation and substitution split over launches for few or large systems: the
// panels run on one workgroup per system (in registers while n - k0 <= 1024, else in global
// memory), the trailing updates and the back substitution on one workgroup per 64 x 64 tile
// (bitwise the same operations as k_dense_solve).
template <int S, int NB = LU_NB>
__global__ __launch_bounds__(256) void k_lu_panel(double2* __restrict__ A, int n, int ld, int k0,
                                                  int* __restrict__ info, int* __restrict__ piv) {
  const int sys = blockIdx.x;
  if (info[sys]) return;
  if constexpr (S > 0) {
    __shared__ PanelSmem psm;
    if (lu_panel_reg<S, NB>(A + int64_t(sys) * n * ld, n, ld, k0, sys, info, psm) && threadIdx.x < NB)
      piv[sys * LU_NB + threadIdx.x] = psm.perm[threadIdx.x];
  } else {
    __shared__ double sv[256];
    __shared__ int si[256];
    (void)lu_panel(A + int64_t(sys) * n * ld, n, ld, k0, sys, info, sv, si);
  }
}

// lu_columns of panel k0 for the columns blockIdx.x * 256 + t, one workgroup per 256 columns
// (after k_lu_panel<S > 0>: L11 from the factored panel, the interchanges from piv)
__global__ __launch_bounds__(256) void k_lu_cols(double2* __restrict__ A, int n, int ld, int k0, int kb,
                                                 const int* __restrict__ info, const int* __restrict__ piv) {
  const int sys = blockIdx.y;
  if (info[sys]) return;
  double2* M = A + int64_t(sys) * n * ld;
  __shared__ double2 L11[LU_NB][LU_NB + 1];
  __shared__ int perm[LU_NB];
  {
    const int r = threadIdx.x / LU_NB, q = threadIdx.x % LU_NB;
    const bool in = r < kb && q < kb;
    const double2 v = M[int64_t(k0 + (in ? r : 0)) * ld + k0 + (in ? q : 0)];
    L11[r][q] = sel2(in, v, make_double2(0, 0));
    if (threadIdx.x < LU_NB) perm[threadIdx.x] = threadIdx.x < kb ? piv[sys * LU_NB + threadIdx.x] : k0;
  }
  __syncthreads();
  lu_columns(M, ld, k0, kb, perm, L11, blockIdx.x * 256 + threadIdx.x, gridDim.x * 256);
}

__global__ __launch_bounds__(256) void k_lu_tiles(double2* __restrict__ A, int n, int ld, int r0, int r1,
                                                  int c0, int c1, int lc, int ur, int kb,
                                                  const int* __restrict__ info) {
  const int sys = blockIdx.y;
  if (info[sys]) return;
  __shared__ double2 Ls[64][LU_NB + 1];
  __shared__ double2 Us[LU_NB][64 + 1];
  const int ntc = (c1 - c0 + 63) / 64;
  const int tr = r0 + (blockIdx.x / ntc) * 64, tc = c0 + (blockIdx.x % ntc) * 64;
  tile_one(A + int64_t(sys) * n * ld, ld, tr, tc, r1, c1, lc, ur, kb, Ls, Us);
}

__global__ __launch_bounds__(256) void k_lu_back_diag(double2* __restrict__ A, int n, int ld, int k0,
                                                      const int* __restrict__ info) {
  const int sys = blockIdx.y;
  if (info[sys]) return;
  __shared__ double2 Ud[LU_NB][LU_NB + 1];
  back_diag(A + int64_t(sys) * n * ld, n, ld, k0, blockIdx.x * 256, gridDim.x * 256, Ud);
}

__global__ void k_info_zero(int* __restrict__ info, int nsys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nsys) info[i] = 0;
}

// out[sys][i][j] = Aug[sys][i][n + j]
__global__ void k_aug_extract(const double2* __restrict__ Aug, int n, int nrhs, double2* __restrict__ out,
                              int nsys) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(nsys) * n * nrhs) return;
  const int64_t sys = e / (int64_t(n) * nrhs);
  const int64_t rem = e - sys * n * nrhs;
  const int i = int(rem / nrhs), j = int(rem - int64_t(i) * nrhs);
  out[e] = Aug[(sys * n + i) * (n + nrhs) + n + j];
}

// Aug[sys] = [A[sys] | I]: A given as nsys blocks of n x n with stride astride (elements) and
// row stride arow
__global__ void k_aug_identity(const double2* __restrict__ A, int64_t astride, int arow, int n,
                               double2* __restrict__ Aug, int nsys) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int ld = 2 * n;
  if (e >= int64_t(nsys) * n * ld) return;
  const int64_t sys = e / (int64_t(n) * ld);
  const int64_t rem = e - sys * n * ld;
  const int i = int(rem / ld), j = int(rem - int64_t(i) * ld);
  Aug[e] = j < n ? A[sys * astride + int64_t(i) * arow + j] : make_double2(j - n == i ? 1.0 : 0.0, 0.0);
}

// Copy the rows of each wirebasket's solution that the wirebasket owns into P [p][i][ncol].
__global__ void k_scatter_P(Geom g, const double2* __restrict__ X, const int* __restrict__ fpos,
                            int nf, const int* __restrict__ owner, double2* __restrict__ P) {
  const int w = blockIdx.x;
  const int I = w / g.nJ, J = w - (w / g.nJ) * g.nJ;
  const int fpw = g.a + g.o, ncol = g.nvcol(), nfd = nf * g.b;
  const double2* Xw = X + int64_t(w) * nfd * (nfd + ncol);
  for (int64_t e = threadIdx.x; e < int64_t(nfd) * ncol; e += blockDim.x) {
    const int rrow = int(e / ncol), col = int(e - int64_t(rrow) * ncol);
    const int fi = rrow / g.b, i = rrow - (rrow / g.b) * g.b;
    const int pos = fpos[fi];
    const int dt = pos / fpw, dx = pos - (pos / fpw) * fpw;
    const int p = wrap_s(g.a * I + dt, g.Lt) * g.Lx + wrap_s(g.a * J + dx, g.Lx);
    if (owner[p] != w) continue;
    // local column (corner, vertex dof) -> the corner's block of bc columns in P's row
    const int c = col / g.bv, j = col - c * g.bv;
    P[(int64_t(p) * g.b + i) * g.ncol() + c * g.bc + j] = Xw[int64_t(rrow) * (nfd + ncol) + nfd + col];
  }
}

// Augmented coarse space, one workgroup per wirebasket w (its owned rows, at most 4 per thread):
// e_j = tv_j - Ptv_j on the rows; Gram-Schmidt in order j = 0..k-1, each projection subtracted
// from the updated vector (v -= q_i (q_i^H v)); q_j goes to P's column bv + j of the rows (corner
// 0, the wirebasket's own node), and q_j^H e_l of every test vector l to the coarse test vector
// tvc_l at node w, dof bv + j.  Sums over the rows are block reductions in a fixed order.
constexpr int kAugRowsPerThread = kAugMaxRows / 256;

__device__ inline double2 block_sum_c(double2 v, double2* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (t < h) red[t] = cadd(red[t], red[t + h]);
    __syncthreads();
  }
  const double2 r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_augment(Geom g, double2* __restrict__ P, const int* __restrict__ rows,
                                                 const int* __restrict__ nrows, int maxrows,
                                                 const double2* __restrict__ tv, const double2* __restrict__ Ptv,
                                                 double2* __restrict__ tvc, int nv, int k, int* __restrict__ info) {
  __shared__ double2 red[256];
  const int w = blockIdx.x;
  const int nr = nrows[w];
  const int64_t nd = g.ndof(), ncd = int64_t(g.nI) * g.nJ * g.bc;
  const int ncol = g.ncol();
  int rr[kAugRowsPerThread];
#pragma unroll
  for (int u = 0; u < kAugRowsPerThread; ++u) {
    const int i = threadIdx.x + u * 256;
    rr[u] = i < nr ? rows[int64_t(w) * maxrows + i] : -1;
  }
  if (threadIdx.x == 0) info[w] = 0;
  for (int j = 0; j < k; ++j) {
    double2 v[kAugRowsPerThread];
#pragma unroll
    for (int u = 0; u < kAugRowsPerThread; ++u)
      v[u] = rr[u] >= 0 ? csub(tv[int64_t(j) * nd + rr[u]], Ptv[int64_t(j) * nd + rr[u]]) : make_double2(0, 0);
    for (int i = 0; i < j; ++i) {
      double2 d = make_double2(0, 0);          // q_i^H v
#pragma unroll
      for (int u = 0; u < kAugRowsPerThread; ++u)
        if (rr[u] >= 0) d = cfmac(P[int64_t(rr[u]) * ncol + g.bv + i], v[u], d);
      d = block_sum_c(d, red);
#pragma unroll
      for (int u = 0; u < kAugRowsPerThread; ++u)
        if (rr[u] >= 0) v[u] = csub(v[u], cmul(P[int64_t(rr[u]) * ncol + g.bv + i], d));
    }
    double2 n2 = make_double2(0, 0);
#pragma unroll
    for (int u = 0; u < kAugRowsPerThread; ++u) n2.x += cabs2(v[u]);
    n2 = block_sum_c(n2, red);
    const double nrm = sqrt(n2.x);
    if (!(nrm > 0)) {
      if (threadIdx.x == 0) info[w] = 1;
      return;
    }
#pragma unroll
    for (int u = 0; u < kAugRowsPerThread; ++u)
      if (rr[u] >= 0) P[int64_t(rr[u]) * ncol + g.bv + j] = make_double2(v[u].x / nrm, v[u].y / nrm);
  }
  // coefficients of every test vector in the wirebasket's basis
  for (int l = 0; l < nv; ++l)
    for (int j = 0; j < k; ++j) {
      double2 d = make_double2(0, 0);
#pragma unroll
      for (int u = 0; u < kAugRowsPerThread; ++u)
        if (rr[u] >= 0)
          d = cfmac(P[int64_t(rr[u]) * ncol + g.bv + j],
                    csub(tv[int64_t(l) * nd + rr[u]], Ptv[int64_t(l) * nd + rr[u]]), d);
      d = block_sum_c(d, red);
      if (threadIdx.x == 0) tvc[int64_t(l) * ncd + int64_t(w) * g.bc + g.bv + j] = d;
    }
}

__device__ inline int corner_node_s(int w, int c, int nI, int nJ) {
  const int I = w / nJ, J = w - (w / nJ) * nJ;
  return ((I + (c >> 1)) % nI) * nJ + (J + (c & 1)) % nJ;
}

// Row scale c of every F row: TESTVEC c = sum_k conj(q_k) w_k / sum_k |q_k|^2 with
// q_k = (P~ w_k|V) at the row; CONST c = 1 / (row sum of P~).
__global__ void k_normalise(Geom g, double2* __restrict__ P, const int* __restrict__ owner,
                            const double2* __restrict__ tv, const double2* __restrict__ tvc,
                            int nv, int mode) {
  const int64_t row = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (row >= g.ndof()) return;
  const int p = int(row / g.b);
  const int w = owner[p];
  if (w < 0) return;
  const int ncol = g.ncol();
  double2* Pr = P + row * ncol;
  double2 c;
  if (mode == 1) {
    double2 sum = make_double2(0, 0);
    for (int col = 0; col < ncol; ++col) sum = cadd(sum, Pr[col]);
    const double den = cabs2(sum);
    c = make_double2(sum.x / den, -sum.y / den);
  } else {
    const int64_t ncd = int64_t(g.nI) * g.nJ * g.bc;
    double2 num = make_double2(0, 0);
    double den = 0;
    for (int k = 0; k < nv; ++k) {
      double2 q = make_double2(0, 0);
      for (int col = 0; col < ncol; ++col) {
        const int cc = col / g.bc, j = col - cc * g.bc;
        q = cfma(Pr[col], tvc[int64_t(k) * ncd + int64_t(corner_node_s(w, cc, g.nI, g.nJ)) * g.bc + j], q);
      }
      num = cfmac(q, tv[int64_t(k) * g.ndof() + row], num);
      den += cabs2(q);
    }
    c = make_double2(num.x / den, num.y / den);
  }
  for (int col = 0; col < ncol; ++col) Pr[col] = cmul(c, Pr[col]);
}

// Probe vectors for the Galerkin operator: e[jj][N][j] = 1 if node N has colour (ct, cx)
// (I mod pt, J mod px) and j == jj.
__global__ void k_probe_make(Geom gc, int pt, int px, int ct, int cx, double2* __restrict__ e) {
  const int64_t nd = int64_t(gc.Lt) * gc.Lx * gc.b;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nd * gc.b) return;
  const int jj = int(i / nd);
  const int64_t d = i - int64_t(jj) * nd;
  const int N = int(d / gc.b), j = int(d - int64_t(N) * gc.b);
  const int I = N / gc.Lx, J = N - (N / gc.Lx) * gc.Lx;
  const bool on = (I % pt == ct) && (J % px == cx) && (j == jj);
  e[i] = make_double2(on ? 1.0 : 0.0, 0.0);
}

// u[jj][N][i] = sum over colour nodes M of A_c[N, M][i][jj]; at most one colour node lies
// within reach 2 of N (periods >= 5), so u gives column jj of the block (N, M).
__global__ void k_probe_extract(Geom gc, int pt, int px, int ct, int cx,
                                const double2* __restrict__ u, double2* __restrict__ out,
                                int dense) {
  const int b = gc.b;
  const int64_t nd = int64_t(gc.Lt) * gc.Lx * b;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nd * b) return;
  const int jj = int(i / nd);
  const int64_t d = i - int64_t(jj) * nd;
  const int N = int(d / b), row = int(d - int64_t(N) * b);
  const int I = N / gc.Lx, J = N - (N / gc.Lx) * gc.Lx;
  const double2 val = u[i];
  if (dense && pt == gc.Lt && px == gc.Lx) {
    const int M = ct * gc.Lx + cx;
    out[(int64_t(N) * b + row) * nd + int64_t(M) * b + jj] = val;
    return;
  }
  int dtf = 99, dxf = 99;
  for (int dt = -2; dt <= 2; ++dt)
    if (wrap_s(I + dt, gc.Lt) % pt == ct) dtf = dt;
  for (int dx = -2; dx <= 2; ++dx)
    if (wrap_s(J + dx, gc.Lx) % px == cx) dxf = dx;
  if (dtf == 99 || dxf == 99) return;
  if (dense) {
    const int M = wrap_s(I + dtf, gc.Lt) * gc.Lx + wrap_s(J + dxf, gc.Lx);
    out[(int64_t(N) * b + row) * nd + int64_t(M) * b + jj] = val;
  } else {
    const int off = (dtf + 2) * 5 + (dxf + 2);
    out[((int64_t(N) * 25 + off) * b + row) * b + jj] = val;
  }
}

__global__ void k_cast_matrix(const double2* __restrict__ A, float2* __restrict__ out, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2(float(A[i].x), float(A[i].y));
}

// ------------------------------------------------------------------------------ launchers

static inline dim3 g1(int64_t n) { return dim3(unsigned((n + 255) / 256)); }

void gather_local(hipStream_t s, const Geom& g, const double2* A, int noff, const int* offs,
                  const int* postab_fpos, int nf, double2* Aug) {
  const int fp = g.fp();
  hipLaunchKernelGGL(k_gather_local, dim3(g.nI * g.nJ), dim3(256), 0, s, g, A, noff, offs,
                     postab_fpos, postab_fpos + fp, nf, Aug);
}

void dense_solve(hipStream_t s, double2* Aug, int n, int nrhs, int nsys, int* info) {
  int* piv = info + nsys;
  const int ld = n + nrhs;
  // many small systems: one workgroup per system for the whole solve; otherwise the panels on
  // one workgroup per system and the trailing updates spread over 64 x 64 tiles
  if (n <= 256 && (nsys >= 32 || n <= 64)) {
    hipLaunchKernelGGL(k_dense_solve, dim3(nsys), dim3(256), 0, s, Aug, n, ld, info);
    return;
  }
  hipLaunchKernelGGL(k_info_zero, dim3((nsys + 63) / 64), dim3(64), 0, s, info, nsys);
  for (int k0 = 0; k0 < n;) {
    // panel rows in registers: up to 1024 rows at width LU_NB, up to 2048 at width 8; beyond,
    // in global memory
    const int rem = n - k0;
    const int kb = std::min(rem > 1024 && rem <= 2048 ? 8 : LU_NB, rem);
    if (rem > 2048) {
      hipLaunchKernelGGL(k_lu_panel<0>, dim3(nsys), dim3(256), 0, s, Aug, n, ld, k0, info, piv);
    } else if (rem > 1024) {
      hipLaunchKernelGGL((k_lu_panel<8, 8>), dim3(nsys), dim3(256), 0, s, Aug, n, ld, k0, info, piv);
    } else {
      switch ((rem + 255) / 256) {
        case 1: hipLaunchKernelGGL(k_lu_panel<1>, dim3(nsys), dim3(256), 0, s, Aug, n, ld, k0, info, piv); break;
        case 2: hipLaunchKernelGGL(k_lu_panel<2>, dim3(nsys), dim3(256), 0, s, Aug, n, ld, k0, info, piv); break;
        case 3: hipLaunchKernelGGL(k_lu_panel<3>, dim3(nsys), dim3(256), 0, s, Aug, n, ld, k0, info, piv); break;
        default: hipLaunchKernelGGL(k_lu_panel<4>, dim3(nsys), dim3(256), 0, s, Aug, n, ld, k0, info, piv);
      }
    }
    if (rem <= 2048 && k0 + kb < ld)
      hipLaunchKernelGGL(k_lu_cols, dim3((ld - k0 - kb + 255) / 256, nsys), dim3(256), 0, s, Aug, n, ld, k0, kb,
                         (const int*)info, (const int*)piv);
    const int r0 = k0 + kb, c0 = k0 + kb;
    if (r0 < n) {
      const int tiles = ((n - r0 + 63) / 64) * ((ld - c0 + 63) / 64);
      hipLaunchKernelGGL(k_lu_tiles, dim3(tiles, nsys), dim3(256), 0, s, Aug, n, ld, r0, n, c0, ld, k0, k0, kb,
                         (const int*)info);
    }
    k0 += kb;
  }
  const int last = ((n - 1) / LU_NB) * LU_NB;
  for (int k0 = last; k0 >= 0; k0 -= LU_NB) {
    const int kb = min(LU_NB, n - k0);
    hipLaunchKernelGGL(k_lu_back_diag, dim3((nrhs + 255) / 256, nsys), dim3(256), 0, s, Aug, n, ld, k0,
                       (const int*)info);
    if (k0 > 0) {
      const int tiles = ((k0 + 63) / 64) * ((ld - n + 63) / 64);
      hipLaunchKernelGGL(k_lu_tiles, dim3(tiles, nsys), dim3(256), 0, s, Aug, n, ld, 0, k0, n, ld, k0, k0, kb,
                         (const int*)info);
    }
  }
}

void aug_extract(hipStream_t s, const double2* Aug, int n, int nrhs, double2* out, int nsys) {
  hipLaunchKernelGGL(k_aug_extract, g1(int64_t(nsys) * n * nrhs), dim3(256), 0, s, Aug, n, nrhs, out, nsys);
}

void aug_identity(hipStream_t s, const double2* A, int64_t astride, int arow, int n, double2* Aug,
                  int nsys) {
  hipLaunchKernelGGL(k_aug_identity, g1(int64_t(nsys) * n * 2 * n), dim3(256), 0, s, A, astride, arow,
                     n, Aug, nsys);
}

void scatter_P(hipStream_t s, const Geom& g, const double2* X, const int* postab_fpos, int nf,
               const int* owner, double2* P) {
  hipLaunchKernelGGL(k_scatter_P, dim3(g.nI * g.nJ), dim3(256), 0, s, g, X, postab_fpos + g.fp(),
                     nf, owner, P);
}

void augment(hipStream_t s, const Geom& g, double2* P, const int* rows, const int* nrows, int maxrows,
             const double2* tv, const double2* Ptv, double2* tvc, int nv, int k, int* info) {
  hipLaunchKernelGGL(k_augment, dim3(g.nI * g.nJ), dim3(256), 0, s, g, P, rows, nrows, maxrows, tv, Ptv, tvc,
                     nv, k, info);
}

void normalise(hipStream_t s, const Geom& g, double2* P, const int* owner, const double2* tv,
               const double2* tvc, int nv, int mode) {
  if (mode == 2) return;
  hipLaunchKernelGGL(k_normalise, g1(g.ndof()), dim3(256), 0, s, g, P, owner, tv, tvc, nv, mode);
}

void probe_make(hipStream_t s, const Geom& gc, int pt, int px, int ct, int cx, double2* e) {
  const int64_t n = int64_t(gc.Lt) * gc.Lx * gc.b * gc.b;
  hipLaunchKernelGGL(k_probe_make, g1(n), dim3(256), 0, s, gc, pt, px, ct, cx, e);
}

void probe_extract(hipStream_t s, const Geom& gc, int pt, int px, int ct, int cx,
                   const double2* u, double2* out, int dense) {
  const int64_t n = int64_t(gc.Lt) * gc.Lx * gc.b * gc.b;
  hipLaunchKernelGGL(k_probe_extract, g1(n), dim3(256), 0, s, gc, pt, px, ct, cx, u, out, dense);
}


void cast_matrix(hipStream_t s, const double2* A, float2* out, int64_t n) {
  hipLaunchKernelGGL(k_cast_matrix, g1(n), dim3(256), 0, s, A, out, n);
}

// y += a x for complex arrays and a real scale (the mass term of the coarse operators)
__global__ void k_axpy_real(double2* __restrict__ y, double a, const double2* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const double2 v = x[i], w = y[i];
    y[i] = make_double2(fma(a, v.x, w.x), fma(a, v.y, w.y));
  }
}

void axpy_real(hipStream_t s, double2* y, double a, const double2* x, int64_t n) {
  hipLaunchKernelGGL(k_axpy_real, g1(n), dim3(256), 0, s, y, a, x, n);
}

}  // namespace amamg
