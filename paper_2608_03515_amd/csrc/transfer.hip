// Transfer kernels between a level and the next coarser one, and the wirebasket classification
// (paper, SM-AMG for LQCD subsection: wirebaskets with vertex / edge / interior points; the
// interpolation of an edge comes from its primary wirebasket, vertices are interpolated by
// the identity; the global interpolator assembles the local ones).
//
// Geometry of level k (grid Lt x Lx, b dofs per node), aggregate size a, overlap o:
//   wirebasket W(I,J) = {(aI + dt, aJ + dx) mod L : 0 <= dt, dx < a + o};
//   point p is a vertex if it lies in 4 wirebaskets, an edge point if in 2, interior if in 1;
//   node (I,J) = the o x o vertices (aI + pt, aJ + px), coarse dof (pt*o + px)*b + q;
//   primary wirebasket of an edge point = the lowest index I * nJ + J containing it.
// Interpolation storage, row-major over fine dofs: P[p][i][c*bc + j], c = 2*ct + cx the corner
// node ((I+ct) mod nI, (J+cx) mod nJ) of p's primary wirebasket, bc = o*o*b (plus the augmented
// dofs on the finest level, which follow the vertex dofs of each node and are nonzero only in
// corner 0, the row's own wirebasket).  Vertex rows are
// the identity and are not stored (left zero).
#include "launch.hpp"

namespace amamg {

__device__ inline int wrapt(int v, int L) { v %= L; return v < 0 ? v + L : v; }

__device__ inline int corner_node(int w, int c, int nI, int nJ) {
  const int I = w / nJ, J = w - (w / nJ) * nJ;
  const int ct = c >> 1, cx = c & 1;
  return ((I + ct) % nI) * nJ + (J + cx) % nJ;
}

// Restriction rc = P^H r in two passes, both fixed-order (deterministic, no atomics).
// Pass 1, one workgroup per (wirebasket W, chunk of W's owned rows): for every interpolation
// column col of W, part[W][chunk][col] = sum over the chunk's rows of conj(P[row][col]) r[row].
// rows[W][k] lists W's owned fine rows (p*b + i) in footprint order (nrows[W] of them); the
// chunk's r values are staged in LDS, lanes run over columns, so each P row is read as one
// contiguous segment.
// Pass 2: rc[N][j] = sum over the 4 wirebaskets W having N as corner c and over their chunks
// of part[W][chunk][c*bc + j], plus r at N's vertices; L lanes per output, xor-reduced.
// Multi-rhs transfer tiles.  A workgroup owns one wirebasket W and a chunk of at most
// `rch` of its owned rows: the interpolation rows of the chunk are staged once in LDS (row
// stride ncol + 1 against bank conflicts) and reused for every right-hand side, which are
// taken `rg` at a time.
struct TileShape { int rch, rg, nchunk; };

__host__ __device__ inline TileShape tile_shape(int ncol, int cs, int maxrows) {
  int rch = 128;
  while (rch > 8 && rch * (ncol + 1) * cs > 32768) rch >>= 1;
  int rg = 16;
  while (rg > 1 && rg * ncol * cs > 16384) rg >>= 1;
  TileShape t;
  t.rch = rch;
  t.rg = rg;
  t.nchunk = (maxrows + rch - 1) / rch;
  return t;
}

// Pass 1 of the restriction: part[r][W][chunk][col] = sum over the chunk's rows of
// conj(P[row][col]) rin_r[row]
template <typename R, typename M, typename Vin>
__global__ __launch_bounds__(256) void k_restrict_partial(const M* __restrict__ P,
                                                          const int* __restrict__ rows,
                                                          const int* __restrict__ nrows,
                                                          int maxrows,
                                                          const Vin* __restrict__ rin,
                                                          cplx<R>* __restrict__ part, Geom g,
                                                          TileShape ts, int nrhs, int64_t stride_f,
                                                          const RhsState* __restrict__ st) {
  using C = cplx<R>;
  extern __shared__ __align__(16) char smem[];
  const int ncol = g.ncol(), pld = ncol + 1;
  C* Pl = reinterpret_cast<C*>(smem);                 // [rch][ncol + 1]
  C* Rl = Pl + ts.rch * pld;                           // [rg][rch]
  int* ri = reinterpret_cast<int*>(Rl + ts.rg * ts.rch);
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int w = bid / ts.nchunk, chunk = bid - (bid / ts.nchunk) * ts.nchunk;
  const int nr = nrows[w];
  const int r0 = chunk * ts.rch, cnt = max(0, min(nr - r0, ts.rch));
  for (int k = threadIdx.x; k < cnt; k += 256) ri[k] = rows[int64_t(w) * maxrows + r0 + k];
  __syncthreads();
  stage<8, 256, M>(cnt * ncol, [&](int e) { return P[int64_t(ri[e / ncol]) * ncol + e % ncol]; },
                   [&](int e, M v) { Pl[(e / ncol) * pld + e % ncol] = cconv<C>(v); });
  const int nW = g.nI * g.nJ;
  for (int g0 = 0; g0 < nrhs; g0 += ts.rg) {
    const int ng = min(ts.rg, nrhs - g0);
    __syncthreads();
    stage<8, 256, Vin>(ng * cnt, [&](int e) { return rin[(g0 + e / cnt) * stride_f + ri[e % cnt]]; },
                       [&](int e, Vin v) {
                         const int rr = e / cnt;
                         Rl[rr * ts.rch + e % cnt] = !st || st[g0 + rr].active ? cconv<C>(v) : czero<R>();
                       });
    __syncthreads();
    for (int q = threadIdx.x; q < ng * ncol; q += 256) {
      const int rr = q / ncol, col = q - (q / ncol) * ncol;
      if (st && !st[g0 + rr].active) continue;
      C acc = czero<R>();
      for (int k = 0; k < cnt; ++k) acc = cfmac(Pl[k * pld + col], Rl[rr * ts.rch + k], acc);
      part[((int64_t(g0 + rr) * nW + w) * ts.nchunk + chunk) * ncol + col] = acc;
    }
  }
}

// Prolongation y = P e (add: y += P e) for every right-hand side.  Workgroup (W, chunk) writes
// the chunk's owned rows of W; chunk 0 also writes the vertex rows of node (I, J) of W, which
// are the identity on corner 0 of W.  A row's sum runs as one chain per corner node, the four
// added in corner order (the order k_prolong_corner4 keeps).
template <typename R, typename M, typename Vin, typename Vout>
__global__ __launch_bounds__(256) void k_prolong(const M* __restrict__ P,
                                                 const int* __restrict__ rows,
                                                 const int* __restrict__ nrows, int maxrows,
                                                 const Vin* __restrict__ e, Vout* __restrict__ y,
                                                 Geom g, TileShape ts, int add, int nrhs,
                                                 int64_t stride_f, int64_t stride_c,
                                                 const RhsState* __restrict__ st) {
  using C = cplx<R>;
  extern __shared__ __align__(16) char smem[];
  const int ncol = g.ncol(), pld = ncol + 1;
  C* Pl = reinterpret_cast<C*>(smem);                 // [rch][ncol + 1]
  C* El = Pl + ts.rch * pld;                           // [rg][ncol]
  int* ri = reinterpret_cast<int*>(El + ts.rg * ncol);
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int w = bid / ts.nchunk, chunk = bid - (bid / ts.nchunk) * ts.nchunk;
  const int I = w / g.nJ, J = w - (w / g.nJ) * g.nJ;
  const int nr = nrows[w];
  const int r0 = chunk * ts.rch, cnt = max(0, min(nr - r0, ts.rch));
  const int nv_rows = chunk == 0 ? g.o * g.o * g.b : 0;     // vertex rows of node (I, J)
  if (cnt == 0 && nv_rows == 0) return;              // no row of W in this chunk
  for (int k = threadIdx.x; k < cnt; k += 256) ri[k] = rows[int64_t(w) * maxrows + r0 + k];
  __syncthreads();
  stage<8, 256, M>(cnt * ncol, [&](int q) { return P[int64_t(ri[q / ncol]) * ncol + q % ncol]; },
                   [&](int q, M v) { Pl[(q / ncol) * pld + q % ncol] = cconv<C>(v); });
  int cn[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) cn[c] = ((I + (c >> 1)) % g.nI) * g.nJ + (J + (c & 1)) % g.nJ;
  const int nout = cnt + nv_rows;
  for (int g0 = 0; g0 < nrhs; g0 += ts.rg) {
    const int ng = min(ts.rg, nrhs - g0);
    __syncthreads();
    stage<8, 256, Vin>(ng * ncol, [&](int q) {
      const int rr = q / ncol, col = q - (q / ncol) * ncol;
      const int c = col / g.bc, j = col - (col / g.bc) * g.bc;
      return e[(g0 + rr) * stride_c + int64_t(cn[c]) * g.bc + j];
    }, [&](int q, Vin v) { El[q] = cconv<C>(v); });
    __syncthreads();
    for (int q = threadIdx.x; q < ng * nout; q += 256) {
      const int rr = q / nout, k = q - (q / nout) * nout;
      if (st && !st[g0 + rr].active) continue;
      C acc;
      int64_t row;
      if (k < cnt) {
        // one chain per corner (columns c bc .. c bc + bc - 1), the four added in corner order
        const C* El_r = El + rr * ncol;
        for (int c = 0; c < 4; ++c) {
          C pc = czero<R>();
          for (int j = c * g.bc; j < (c + 1) * g.bc; ++j) pc = cfma(Pl[k * pld + j], El_r[j], pc);
          acc = c == 0 ? pc : cadd(acc, pc);
        }
        row = ri[k];
      } else {
        const int v = k - cnt;                       // (pt*o + px)*b + q of node (I, J)
        const int qq = v % g.b, pp = v / g.b;
        const int pt = pp / g.o, px = pp - (pp / g.o) * g.o;
        row = int64_t((g.a * I + pt) * g.Lx + (g.a * J + px)) * g.b + qq;
        acc = El[rr * ncol + v];                     // corner 0 is node (I, J)
      }
      Vout* yr = y + (g0 + rr) * stride_f;
      if (add) acc = cadd(acc, cconv<C>(yr[row]));
      yr[row] = cconv<Vout>(acc);
    }
  }
}

// Register-tiled transfer for NCOL interpolation columns (NCOL divides 64: the fine level of
// overlap 1 and 2), right-hand sides 32 per pass.  The generic kernels above read two LDS values
// per complex multiply-add; these read each interpolation value once per row for several
// right-hand sides and take the right-hand-side values as wave-wide broadcasts.
// Tile shapes (measured at the 256^2, a = 8, o = 2 fine level): small enough for several
// workgroups per compute unit, which hide the row gather's latency.
template <typename R, int NCOL> struct TiledRows {
  static constexpr int RESTRICT = sizeof(R) == 4 ? 60 : 30;    // rows per restriction chunk
  static constexpr int PROLONG = sizeof(R) == 4 ? 64 : 32;     // rows per prolongation chunk
  // right-hand sides per pass (the restriction's lane tiling needs 4 * 64 / NCOL at least)
  static constexpr int RHS_R = NCOL == 8 ? 32 : (sizeof(R) == 4 ? 32 : 16);
  static constexpr int RHS_P = sizeof(R) == 4 ? 32 : 16;
};
__host__ __device__ inline bool tiled_cols(int ncol) { return ncol == 8 || ncol == 32; }

// Restriction pass 1 (same partial layout as k_restrict_partial): lane (sub, col) of wave wv
// accumulates conj(P[k][col]) r[k] for the RB right-hand sides wv*SUB*RB + sub + SUB*j.
template <int NCOL, int RCH, int NR, typename R, typename M, typename Vin>
__global__ __launch_bounds__(256) void k_restrict_partial_tiled(
    const M* __restrict__ P, const int* __restrict__ rows, const int* __restrict__ nrows, int maxrows,
    const Vin* __restrict__ rin, cplx<R>* __restrict__ part, int nW, int nchunk, int nrhs,
    int64_t stride_f, const RhsState* __restrict__ st) {
  using C = cplx<R>;
  constexpr int SUB = 64 / NCOL, RB = NR / (4 * SUB), RS = RCH + 1;
  static_assert(RB >= 1 && 4 * SUB * RB == NR, "lane tiling must cover the pass");
  __shared__ C Pl[RCH * NCOL];
  __shared__ C Rl[NR * RS];             // row stride RCH + 1 against bank conflicts
  __shared__ int ri[RCH];
  __shared__ int live[NR];
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int w = bid / nchunk, chunk = bid - (bid / nchunk) * nchunk;
  const int r0 = chunk * RCH, cnt = max(0, min(nrows[w] - r0, RCH));
  for (int k = threadIdx.x; k < cnt; k += 256) ri[k] = rows[int64_t(w) * maxrows + r0 + k];
  __syncthreads();
  stage<8, 256, M>(cnt * NCOL, [&](int q) { return P[int64_t(ri[q / NCOL]) * NCOL + q % NCOL]; },
                   [&](int q, M v) { Pl[q] = cconv<C>(v); });
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane % NCOL, sub = lane / NCOL;
  for (int g0 = 0; g0 < nrhs; g0 += NR) {
    const int ng = min(NR, nrhs - g0);
    __syncthreads();
    for (int rr = threadIdx.x; rr < NR; rr += 256) live[rr] = rr < ng && (!st || st[g0 + rr].active);
    __syncthreads();
    // the fetch only loads (from a clamped address); conversion and masking happen at the store,
    // so that the loads of a batch stay in flight together
    stage<8, 256, Vin>(NR * cnt, [&](int q) {
      const int rr = q / cnt, k = q - rr * cnt;
      return rin[(g0 + (live[rr] ? rr : 0)) * stride_f + ri[k]];
    }, [&](int q, Vin v) {
      const int rr = q / cnt, k = q - rr * cnt;
      Rl[rr * RS + k] = live[rr] ? cconv<C>(v) : czero<R>();
    });
    __syncthreads();
    C acc[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) acc[j] = czero<R>();
    const int rb0 = wv * SUB * RB + sub;
    for (int k = 0; k < cnt; ++k) {
      const C pk = Pl[k * NCOL + col];
#pragma unroll
      for (int j = 0; j < RB; ++j) acc[j] = cfmac(pk, Rl[(rb0 + SUB * j) * RS + k], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int rr = rb0 + SUB * j;
      if (live[rr])
        part[((int64_t(g0 + rr) * nW + w) * nchunk + chunk) * NCOL + col] = acc[j];
    }
  }
}

// Prolongation y = P e (add: y += P e): thread (row k, h) keeps interpolation row k in registers
// and serves the right-hand sides rr = h, h + H, ... of each pass; all lanes of a wave share rr,
// so the coarse values are broadcast LDS reads.  Chunk 0 also writes the vertex rows of node
// (I, J) (identity on corner 0).
template <int NCOL, int RCH, int NR, typename R, typename M, typename Vin, typename Vout>
__global__ __launch_bounds__(256) void k_prolong_tiled(
    const M* __restrict__ P, const int* __restrict__ rows, const int* __restrict__ nrows, int maxrows,
    const Vin* __restrict__ e, Vout* __restrict__ y, Geom g, int nchunk, int add, int nrhs,
    int64_t stride_f, int64_t stride_c, const RhsState* __restrict__ st) {
  using C = cplx<R>;
  constexpr int H = 256 / RCH, PS = NCOL + 1;
  __shared__ C Pl[RCH * PS];            // row stride NCOL + 1 against bank conflicts
  __shared__ C El[NR * NCOL];
  __shared__ int ri[RCH];
  __shared__ int live[NR];              // this pass's active flags, read once per workgroup
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int w = bid / nchunk, chunk = bid - (bid / nchunk) * nchunk;
  const int I = w / g.nJ, J = w - (w / g.nJ) * g.nJ;
  const int r0 = chunk * RCH, cnt = max(0, min(nrows[w] - r0, RCH));
  const int nv_rows = chunk == 0 ? g.o * g.o * g.b : 0;
  if (cnt == 0 && nv_rows == 0) return;              // no row of W in this chunk
  for (int k = threadIdx.x; k < cnt; k += 256) ri[k] = rows[int64_t(w) * maxrows + r0 + k];
  __syncthreads();
  stage<8, 256, M>(cnt * NCOL, [&](int q) { return P[int64_t(ri[q / NCOL]) * NCOL + q % NCOL]; },
                   [&](int q, M v) { Pl[(q / NCOL) * PS + q % NCOL] = cconv<C>(v); });
  __syncthreads();
  const int k = threadIdx.x % RCH, h = threadIdx.x / RCH;
  C pr[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) pr[c] = k < cnt ? Pl[k * PS + c] : czero<R>();
  int cn[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) cn[c] = ((I + (c >> 1)) % g.nI) * g.nJ + (J + (c & 1)) % g.nJ;
  const int row = k < cnt ? ri[k] : 0;
  for (int g0 = 0; g0 < nrhs; g0 += NR) {
    const int ng = min(NR, nrhs - g0);
    __syncthreads();
    stage<8, 256, Vin>(NR * NCOL, [&](int q) {
      const int rr = q / NCOL, col = q % NCOL;
      const int c = col / g.bc, j = col - (col / g.bc) * g.bc;
      return e[(g0 + (rr < ng ? rr : 0)) * stride_c + int64_t(cn[c]) * g.bc + j];
    }, [&](int q, Vin v) { El[q] = q / NCOL < ng ? cconv<C>(v) : czero<R>(); });
    for (int rr = threadIdx.x; rr < NR; rr += 256) live[rr] = rr < ng && (!st || st[g0 + rr].active);
    __syncthreads();
    if (k < cnt)
      for (int rr = h; rr < ng; rr += H) {
        if (!live[rr]) continue;
        C acc = czero<R>();
#pragma unroll
        for (int c = 0; c < NCOL; ++c) acc = cfma(pr[c], El[rr * NCOL + c], acc);
        Vout* yr = y + (g0 + rr) * stride_f;
        if (add) acc = cadd(acc, cconv<C>(yr[row]));
        yr[row] = cconv<Vout>(acc);
      }
    for (int q = threadIdx.x; q < ng * nv_rows; q += 256) {
      const int rr = q / nv_rows, v = q - rr * nv_rows;   // (pt*o + px)*b + qq of node (I, J)
      if (!live[rr]) continue;
      const int qq = v % g.b, pp = v / g.b;
      const int pt = pp / g.o, px = pp - (pp / g.o) * g.o;
      const int64_t vrow = int64_t((g.a * I + pt) * g.Lx + (g.a * J + px)) * g.b + qq;
      C acc = El[rr * NCOL + v];
      Vout* yr = y + (g0 + rr) * stride_f;
      if (add) acc = cadd(acc, cconv<C>(yr[vrow]));
      yr[vrow] = cconv<Vout>(acc);
    }
  }
}

// Transfers of a few right-hand sides (up to kRowsRhs) on the levels served by the tiled
// kernels.  The tiled kernels stage interpolation rows in LDS for passes of 16 or 32 right-hand
// sides; with one right-hand side most of their lanes idle while each chunk pays the staging's
// round trips.  These read the interpolation straight into registers, one thread per output
// value, and repeat the tiled kernels' arithmetic exactly: the same conversions and the same
// multiply-add chains in the same order (prolongation: over a row's columns; restriction: over
// the rows of a chunk of the same length), so a right-hand side gets bitwise the same result in
// every batch.
constexpr int kRowsRhs = 4;

// one interpolation row into registers, converted to the compute type; FP32 rows are read as
// 16-byte pairs (rows are NCOL * 8 bytes long, NCOL even, and start 16-byte aligned)
template <int NCOL, typename C>
__device__ inline void load_row(const double2* __restrict__ p, C (&out)[NCOL]) {
  double2 v[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) v[c] = p[c];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) out[c] = cconv<C>(v[c]);
}
template <int NCOL, typename C>
__device__ inline void load_row(const float2* __restrict__ p, C (&out)[NCOL]) {
  static_assert(NCOL % 2 == 0, "rows of float pairs");
  float4 v[NCOL / 2];
  const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int c = 0; c < NCOL / 2; ++c) v[c] = q[c];
#pragma unroll
  for (int c = 0; c < NCOL / 2; ++c) {
    out[2 * c] = cconv<C>(make_float2(v[c].x, v[c].y));
    out[2 * c + 1] = cconv<C>(make_float2(v[c].z, v[c].w));
  }
}

// Prolongation, one wave per (wirebasket W, chunk of 64 owned rows): lane k holds row k's
// interpolation and serves the right-hand sides in turn; the coarse values of W's corners are
// staged once in LDS.  Chunk 0 also writes the vertex rows of node (I, J) (identity on corner 0).
template <int NCOL, typename R, typename M, typename Vin, typename Vout>
__global__ __launch_bounds__(64) void k_prolong_rows(
    const M* __restrict__ P, const int* __restrict__ rows, const int* __restrict__ nrows, int maxrows,
    const Vin* __restrict__ e, Vout* __restrict__ y, Geom g, int nchunk, int add, int nrhs,
    int64_t stride_f, int64_t stride_c, const RhsState* __restrict__ st) {
  using C = cplx<R>;
  __shared__ C El[kRowsRhs * NCOL];
  __shared__ int live[kRowsRhs];
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int w = bid / nchunk, chunk = bid - (bid / nchunk) * nchunk;
  const int I = w / g.nJ, J = w - (w / g.nJ) * g.nJ;
  const int k = chunk * 64 + int(threadIdx.x);
  const bool own = k < nrows[w];
  const int row = own ? rows[int64_t(w) * maxrows + k] : 0;
  C pr[NCOL];
  load_row<NCOL>(P + int64_t(row) * NCOL, pr);
  int cn[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) cn[c] = ((I + (c >> 1)) % g.nI) * g.nJ + (J + (c & 1)) % g.nJ;
  for (int q = threadIdx.x; q < kRowsRhs * NCOL; q += 64) {
    const int rr = q / NCOL, col = q % NCOL;
    const int c = col / g.bc, j = col - (col / g.bc) * g.bc;
    const Vin v = e[(rr < nrhs ? rr : 0) * stride_c + int64_t(cn[c]) * g.bc + j];
    El[q] = rr < nrhs ? cconv<C>(v) : czero<R>();
  }
  if (threadIdx.x < kRowsRhs) live[threadIdx.x] = int(threadIdx.x) < nrhs && (!st || st[threadIdx.x].active);
  __syncthreads();
  if (own)
    for (int rr = 0; rr < nrhs; ++rr) {
      if (!live[rr]) continue;
      C acc = czero<R>();
#pragma unroll
      for (int c = 0; c < NCOL; ++c) acc = cfma(pr[c], El[rr * NCOL + c], acc);
      Vout* yr = y + rr * stride_f;
      if (add) acc = cadd(acc, cconv<C>(yr[row]));
      yr[row] = cconv<Vout>(acc);
    }
  const int nv_rows = chunk == 0 ? g.o * g.o * g.b : 0;
  for (int q = threadIdx.x; q < nrhs * nv_rows; q += 64) {
    const int rr = q / nv_rows, v = q - rr * nv_rows;      // (pt*o + px)*b + qq of node (I, J)
    if (!live[rr]) continue;
    const int qq = v % g.b, pp = v / g.b;
    const int pt = pp / g.o, px = pp - (pp / g.o) * g.o;
    const int64_t vrow = int64_t((g.a * I + pt) * g.Lx + (g.a * J + px)) * g.b + qq;
    C acc = El[rr * NCOL + v];
    Vout* yr = y + rr * stride_f;
    if (add) acc = cadd(acc, cconv<C>(yr[vrow]));
    yr[vrow] = cconv<Vout>(acc);
  }
}

// Prolongation of up to kRowsRhs right-hand sides for the generic kernel's levels with BC
// degrees of freedom per corner node (128 interpolation columns: level 1 of a = 8, o = 2 in
// FP64).  Four lanes per row, one per corner node: lane c keeps the row's BC values of corner c
// in registers and runs k_prolong's chain for that corner; lane 0 of the four adds the four
// chains in corner order.  Workgroup (W, chunk of 64 owned rows); chunk 0 also writes the vertex
// rows of node (I, J).
template <int BC, typename R, typename M, typename Vin, typename Vout>
__global__ __launch_bounds__(256) void k_prolong_corner4(
    const M* __restrict__ P, const int* __restrict__ rows, const int* __restrict__ nrows, int maxrows,
    const Vin* __restrict__ e, Vout* __restrict__ y, Geom g, int nchunk, int add, int nrhs,
    int64_t stride_f, int64_t stride_c, const RhsState* __restrict__ st) {
  using C = cplx<R>;
  constexpr int NCOL = 4 * BC;
  __shared__ C El[kRowsRhs * NCOL];
  __shared__ int live[kRowsRhs];
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int w = bid / nchunk, chunk = bid - (bid / nchunk) * nchunk;
  const int I = w / g.nJ, J = w - (w / g.nJ) * g.nJ;
  const int c = threadIdx.x & 3, k = chunk * 64 + int(threadIdx.x >> 2);
  const bool own = k < nrows[w];
  const int row = own ? rows[int64_t(w) * maxrows + k] : 0;
  C pr[BC];
  {
    M v[BC];
    const M* pc = P + int64_t(row) * NCOL + c * BC;
#pragma unroll
    for (int j = 0; j < BC; ++j) v[j] = pc[j];
#pragma unroll
    for (int j = 0; j < BC; ++j) pr[j] = cconv<C>(v[j]);
  }
  int cn[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) cn[q] = ((I + (q >> 1)) % g.nI) * g.nJ + (J + (q & 1)) % g.nJ;
  for (int q = threadIdx.x; q < kRowsRhs * NCOL; q += 256) {
    const int rr = q / NCOL, col = q % NCOL;
    const int cc = col / BC, j = col - cc * BC;
    const Vin v = e[(rr < nrhs ? rr : 0) * stride_c + int64_t(cn[cc]) * BC + j];
    El[q] = rr < nrhs ? cconv<C>(v) : czero<R>();
  }
  if (threadIdx.x < kRowsRhs) live[threadIdx.x] = int(threadIdx.x) < nrhs && (!st || st[threadIdx.x].active);
  __syncthreads();
  for (int rr = 0; rr < nrhs; ++rr) {
    if (!live[rr]) continue;                                 // uniform over the workgroup
    C pc = czero<R>();
#pragma unroll
    for (int j = 0; j < BC; ++j) pc = cfma(pr[j], El[rr * NCOL + c * BC + j], pc);
    const int l0 = threadIdx.x & 63 & ~3;
    C q1, q2, q3;
    q1.x = __shfl(pc.x, l0 + 1); q1.y = __shfl(pc.y, l0 + 1);
    q2.x = __shfl(pc.x, l0 + 2); q2.y = __shfl(pc.y, l0 + 2);
    q3.x = __shfl(pc.x, l0 + 3); q3.y = __shfl(pc.y, l0 + 3);
    if (c == 0 && own) {
      C acc = cadd(cadd(cadd(pc, q1), q2), q3);
      Vout* yr = y + rr * stride_f;
      if (add) acc = cadd(acc, cconv<C>(yr[row]));
      yr[row] = cconv<Vout>(acc);
    }
  }
  const int nv_rows = chunk == 0 ? g.o * g.o * g.b : 0;
  for (int q = threadIdx.x; q < nrhs * nv_rows; q += 256) {
    const int rr = q / nv_rows, v = q - rr * nv_rows;      // (pt*o + px)*b + qq of node (I, J)
    if (!live[rr]) continue;
    const int qq = v % g.b, pp = v / g.b;
    const int pt = pp / g.o, px = pp - (pp / g.o) * g.o;
    const int64_t vrow = int64_t((g.a * I + pt) * g.Lx + (g.a * J + px)) * g.b + qq;
    C acc = El[rr * NCOL + v];
    Vout* yr = y + rr * stride_f;
    if (add) acc = cadd(acc, cconv<C>(yr[vrow]));
    yr[vrow] = cconv<Vout>(acc);
  }
}

// Restriction pass 1 (same partial layout and chunks as k_restrict_partial_tiled): thread
// (chunk, col) accumulates conj(P[k][col]) r[k] over the chunk's RCH rows for NS right-hand
// sides; a workgroup serves 8 chunks.  The chunks' row indices and r values are staged in LDS
// while the interpolation values load into registers.
constexpr int kRowsChunks = 8;
template <int NCOL, int RCH, int NS, typename R, typename M, typename Vin>
__global__ __launch_bounds__(kRowsChunks * NCOL) void k_restrict_rows(
    const M* __restrict__ P, const int* __restrict__ rows, const int* __restrict__ nrows, int maxrows,
    const Vin* __restrict__ rin, cplx<R>* __restrict__ part, int nW, int nchunk, int nrhs,
    int64_t stride_f, const RhsState* __restrict__ st) {
  using C = cplx<R>;
  constexpr int CPB = kRowsChunks, NT = CPB * NCOL;        // chunks per workgroup, threads
  __shared__ int ri[CPB * RCH];
  __shared__ C Rl[NS * CPB * RCH];
  __shared__ int cnts[CPB];
  const int npair = nW * nchunk, gc0 = blockIdx.x * CPB;
  if (threadIdx.x < CPB) {
    const int gc = gc0 + int(threadIdx.x);
    const int w = gc / nchunk, r0 = (gc - w * nchunk) * RCH;
    cnts[threadIdx.x] = gc < npair ? max(0, min(nrows[w] - r0, RCH)) : 0;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < CPB * RCH; q += NT) {
    const int cb = q / RCH, k = q - cb * RCH, gc = gc0 + cb;
    const int w = gc / nchunk, r0 = (gc - w * nchunk) * RCH;
    ri[q] = k < cnts[cb] ? rows[int64_t(w) * maxrows + r0 + k] : 0;
  }
  __syncthreads();
  const int cb = threadIdx.x / NCOL, col = threadIdx.x % NCOL;
  const int gc = gc0 + cb, cnt = cnts[cb];
  M pv[RCH];
#pragma unroll
  for (int k = 0; k < RCH; ++k) pv[k] = P[int64_t(ri[cb * RCH + k]) * NCOL + col];
  // r values of the workgroup's rows (the fetch only loads; masking happens at the store)
  for (int q = threadIdx.x; q < NS * CPB * RCH; q += NT) {
    const int rr = q / (CPB * RCH), kq = q - rr * (CPB * RCH);
    const bool lv = rr < nrhs && (!st || st[rr].active);
    const Vin v = rin[(lv ? rr : 0) * stride_f + ri[kq]];
    Rl[q] = lv ? cconv<C>(v) : czero<R>();
  }
  __syncthreads();
  if (gc >= npair) return;
  const int w = gc / nchunk, chunk = gc - w * nchunk;
  C acc[NS];
#pragma unroll
  for (int rr = 0; rr < NS; ++rr) acc[rr] = czero<R>();
#pragma unroll
  for (int k = 0; k < RCH; ++k) {
    if (k < cnt) {
      const C pk = cconv<C>(pv[k]);
#pragma unroll
      for (int rr = 0; rr < NS; ++rr) acc[rr] = cfmac(pk, Rl[rr * CPB * RCH + cb * RCH + k], acc[rr]);
    }
  }
#pragma unroll
  for (int rr = 0; rr < NS; ++rr)
    if (rr < nrhs && (!st || st[rr].active))
      part[((int64_t(rr) * nW + w) * nchunk + chunk) * NCOL + col] = acc[rr];
}

// Matrix-core transfers (FP32, NCOL = 128 interpolation columns, NR = 64 or 32 right-hand sides
// per workgroup).  Per wirebasket the transfer is a dense complex product between the chunk's
// interpolation rows and the right-hand sides; it runs as real 16x16x4 FP32 MFMA tiles
// (v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[4 (l / 16) + i][l % 16], i < 4), four real products per complex one.  D is oriented with the
// right-hand side as its row index, so a lane's results run along interpolation columns
// (restriction) or fine rows (prolongation) and the stores are contiguous.  Wave w owns the
// right-hand sides 16 (w % (NR / 16)) .. + 15 of the workgroup's group and, with NR = 32, half of
// the column (restriction) or row (prolongation) tiles.  Each result is one MFMA chain over the
// same operands in the same order whatever NR, so batches of up to 32 right-hand sides (NR = 32,
// no padding of a 64-wide tile) and larger ones give a right-hand side bitwise the same result.
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
__device__ inline mfma_f4 mfma16(float a, float b, mfma_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <int NCOL> struct MfmaRows;                   // fine rows per chunk
// prolongation rows per chunk: 64 with 64-rhs tiles, 32 with 32-rhs tiles (which then keep
// two workgroups per compute unit); a row's result does not depend on its chunk
template <> struct MfmaRows<128> { static constexpr int RESTRICT = 32, PROLONG = 64, PROLONG32 = 32; };
constexpr int kMfmaRhs = 64;
// The matrix-core path serves 128 columns (coarse levels of a = 8, o = 2); with 32 columns (the
// fine level) the register-tiled kernels above are faster: their smaller LDS footprint keeps
// more workgroups per compute unit to hide the row gather, which dominates there.
__host__ __device__ inline bool mfma_cols(int ncol) { return ncol == 128; }

// Restriction pass 1 (same partial layout as k_restrict_partial):
// D[rhs][col] = sum over the chunk's rows of r_rhs[row] conj(P[row][col]).
template <int NCOL, int RCH, typename Vin, int NR>
__global__ __launch_bounds__(256) void k_restrict_mfma(
    const float2* __restrict__ P, const int* __restrict__ rows, const int* __restrict__ nrows, int maxrows,
    const Vin* __restrict__ rin, float2* __restrict__ part, int nW, int nchunk, int nrhs, int64_t stride_f,
    const RhsState* __restrict__ st) {
  constexpr int WR = NR / 16, WS = 4 / WR;              // rhs tiles, column-tile splits
  static_assert(RCH % 4 == 0 && NCOL % (16 * WS) == 0 && WR * WS == 4, "tile shape");
  constexpr int RS = RCH + 1, PS = NCOL + 1, CT = NCOL / (16 * WS);
  __shared__ float2 Pl[RCH * PS];
  __shared__ float2 Rl[NR * RS];
  __shared__ int ri[RCH];
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int w = bid / nchunk, chunk = bid - (bid / nchunk) * nchunk;
  const int g0 = blockIdx.y * NR, ng = min(NR, nrhs - g0);
  const int r0 = chunk * RCH, cnt = max(0, min(nrows[w] - r0, RCH));
  __shared__ int live[NR];
  for (int k = threadIdx.x; k < RCH; k += 256) ri[k] = k < cnt ? rows[int64_t(w) * maxrows + r0 + k] : 0;
  for (int rr = threadIdx.x; rr < NR; rr += 256) live[rr] = rr < ng && (!st || st[g0 + rr].active);
  __syncthreads();
  // the fetches only load, from valid addresses (ri[k] = 0 past the chunk's rows, rhs 0 of the
  // group for dead ones); conversion and masking happen at the store, so that the loads of a
  // batch stay in flight together
  stage<8, 256, float2>(RCH * NCOL, [&](int q) { return P[int64_t(ri[q / NCOL]) * NCOL + q % NCOL]; },
                        [&](int q, float2 v) { Pl[(q / NCOL) * PS + q % NCOL] = q / NCOL < cnt ? v : make_float2(0.f, 0.f); });
  stage<8, 256, Vin>(NR * RCH, [&](int q) {
    const int rr = q / RCH, k = q - (q / RCH) * RCH;
    return rin[(g0 + (live[rr] ? rr : 0)) * stride_f + ri[k]];
  }, [&](int q, Vin v) {
    const int rr = q / RCH, k = q - (q / RCH) * RCH;
    Rl[rr * RS + k] = live[rr] && k < cnt ? cconv<float2>(v) : make_float2(0.f, 0.f);
  });
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, lr = lane & 15, lk = lane >> 4;
  const int rt = wv % WR, c0 = (wv / WR) * CT * 16;          // this wave's rhs tile, first column
  mfma_f4 re[CT], im[CT];
#pragma unroll
  for (int t = 0; t < CT; ++t) re[t] = im[t] = mfma_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int kk = 0; kk < RCH; kk += 4) {
    const float2 a = Rl[(rt * 16 + lr) * RS + kk + lk];            // A[rhs][row] = r
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const float2 b = Pl[(kk + lk) * PS + c0 + t * 16 + lr];       // B[row][col] = P
      re[t] = mfma16(a.x, b.x, re[t]);
      re[t] = mfma16(a.y, b.y, re[t]);
      im[t] = mfma16(a.y, b.x, im[t]);
      im[t] = mfma16(-a.x, b.y, im[t]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rr = rt * 16 + 4 * lk + i;
    if (live[rr]) {
      float2* out = part + ((int64_t(g0 + rr) * nW + w) * nchunk + chunk) * NCOL + c0 + lr;
#pragma unroll
      for (int t = 0; t < CT; ++t) out[t * 16] = make_float2(re[t][i], im[t][i]);
    }
  }
}

// Prolongation y = P e (add: y += P e): D[rhs][row] = sum_col e_rhs[col] P[row][col] over the
// chunk's rows; chunk 0 also writes the vertex rows of node (I, J) (identity on corner 0).
template <int NCOL, int RCH, int NR>
__global__ __launch_bounds__(256) void k_prolong_mfma(
    const float2* __restrict__ P, const int* __restrict__ rows, const int* __restrict__ nrows, int maxrows,
    const float2* __restrict__ e, float2* __restrict__ y, Geom g, int nchunk, int add, int nrhs,
    int64_t stride_f, int64_t stride_c, const RhsState* __restrict__ st) {
  constexpr int WR = NR / 16, WS = 4 / WR;              // rhs tiles, row-tile splits
  static_assert(RCH % (16 * WS) == 0 && NCOL % 4 == 0 && WR * WS == 4, "tile shape");
  constexpr int PS = NCOL + 1, ES = NCOL + 1, RT = RCH / (16 * WS);
  __shared__ float2 Pl[RCH * PS];
  __shared__ float2 El[NR * ES];
  __shared__ int ri[RCH];
  __shared__ int live[NR];
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int w = bid / nchunk, chunk = bid - (bid / nchunk) * nchunk;
  const int I = w / g.nJ, J = w - (w / g.nJ) * g.nJ;
  const int g0 = blockIdx.y * NR, ng = min(NR, nrhs - g0);
  const int r0 = chunk * RCH, cnt = max(0, min(nrows[w] - r0, RCH));
  const int nv_rows = chunk == 0 ? g.o * g.o * g.b : 0;
  if (cnt == 0 && nv_rows == 0) return;              // no row of W in this chunk
  for (int k = threadIdx.x; k < RCH; k += 256) ri[k] = k < cnt ? rows[int64_t(w) * maxrows + r0 + k] : 0;
  for (int rr = threadIdx.x; rr < NR; rr += 256) live[rr] = rr < ng && (!st || st[g0 + rr].active);
  __syncthreads();
  stage<8, 256, float2>(RCH * NCOL, [&](int q) { return P[int64_t(ri[q / NCOL]) * NCOL + q % NCOL]; },
                        [&](int q, float2 v) { Pl[(q / NCOL) * PS + q % NCOL] = q / NCOL < cnt ? v : make_float2(0.f, 0.f); });
  int cn[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) cn[c] = ((I + (c >> 1)) % g.nI) * g.nJ + (J + (c & 1)) % g.nJ;
  stage<8, 256, float2>(NR * NCOL, [&](int q) {
    const int rr = q / NCOL, col = q - (q / NCOL) * NCOL;
    const int c = col / g.bc, j = col - (col / g.bc) * g.bc;
    return e[(g0 + (rr < ng ? rr : 0)) * stride_c + int64_t(cn[c]) * g.bc + j];
  }, [&](int q, float2 v) { El[(q / NCOL) * ES + q % NCOL] = q / NCOL < ng ? v : make_float2(0.f, 0.f); });
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, lr = lane & 15, lk = lane >> 4;
  const int rt = wv % WR, k0 = (wv / WR) * RT * 16;           // this wave's rhs tile, first row
  mfma_f4 re[RT], im[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) re[t] = im[t] = mfma_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int kc = 0; kc < NCOL; kc += 4) {
    const float2 a = El[(rt * 16 + lr) * ES + kc + lk];            // A[rhs][col] = e
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const float2 b = Pl[(k0 + t * 16 + lr) * PS + kc + lk];       // B[col][row] = P[row][col]
      re[t] = mfma16(a.x, b.x, re[t]);
      re[t] = mfma16(-a.y, b.y, re[t]);
      im[t] = mfma16(a.x, b.y, im[t]);
      im[t] = mfma16(a.y, b.x, im[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int k = k0 + t * 16 + lr;
    if (k >= cnt) continue;
    const int row = ri[k];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = rt * 16 + 4 * lk + i;
      if (!live[rr]) continue;
      float2* yr = y + (g0 + rr) * stride_f;
      float2 v = make_float2(re[t][i], im[t][i]);
      if (add) v = cadd(v, yr[row]);
      yr[row] = v;
    }
  }
  for (int q = threadIdx.x; q < ng * nv_rows; q += 256) {
    const int rr = q / nv_rows, v = q - rr * nv_rows;   // (pt*o + px)*b + qq of node (I, J)
    if (!live[rr]) continue;
    const int qq = v % g.b, pp = v / g.b;
    const int pt = pp / g.o, px = pp - (pp / g.o) * g.o;
    const int64_t vrow = int64_t((g.a * I + pt) * g.Lx + (g.a * J + px)) * g.b + qq;
    float2 acc = El[rr * ES + v];
    float2* yr = y + (g0 + rr) * stride_f;
    if (add) acc = cadd(acc, yr[vrow]);
    yr[vrow] = acc;
  }
}

template <typename R, typename Vin, typename Vout, int CHL>
__global__ __launch_bounds__(256) void k_restrict_gather(const cplx<R>* __restrict__ part,
                                                         const Vin* __restrict__ rin,
                                                         Vout* __restrict__ rc, Geom g, int nchunk,
                                                         int lanes, int64_t stride_f,
                                                         int64_t stride_c,
                                                         const RhsState* __restrict__ st) {
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  using C = cplx<R>;
  const int64_t gid = (int64_t(blockIdx.x) * 256 + threadIdx.x) / lanes;
  const int ln = threadIdx.x % lanes;
  const int nW = g.nI * g.nJ;
  const bool live = gid < int64_t(nW) * g.bc;
  const int64_t gg = live ? gid : 0;
  const int N = int(gg / g.bc), j = int(gg - int64_t(N) * g.bc);
  const int I = N / g.nJ, J = N - (N / g.nJ) * g.nJ;
  const int ncol = g.ncol();
  // all loads first (from valid addresses: chunk 0 past the end), then the sums in the order
  // corner, chunk, so that the loads are in flight together
  // the node's vertex dofs also take r at the vertex (identity rows); the augmented dofs after
  // them (j >= bv) only the wirebasket sums
  const bool vert = j < g.bv;
  const int jv = vert ? j : 0;
  const int q = jv % g.b, pp = jv / g.b;
  const int pt = pp / g.o, px = pp - (pp / g.o) * g.o;
  const int p = (g.a * I + pt) * g.Lx + (g.a * J + px);
  const Vin rv = rin[r * stride_f + int64_t(p) * g.b + q];
  const C* pw[4];
  C pv[4][CHL];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int WI = I - (c >> 1), WJ = J - (c & 1);
    const int w = (WI < 0 ? WI + g.nI : WI) * g.nJ + (WJ < 0 ? WJ + g.nJ : WJ);
    pw[c] = part + (int64_t(r) * nW + w) * nchunk * ncol + c * g.bc + j;
#pragma unroll
    for (int u = 0; u < CHL; ++u) {
      const int ch = ln + u * lanes;
      pv[c][u] = pw[c][int64_t(ch < nchunk ? ch : 0) * ncol];
    }
  }
  C sum = czero<R>();
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int u = 0; u < CHL; ++u)
      if (ln + u * lanes < nchunk) sum = cadd(sum, pv[c][u]);
    for (int ch = ln + CHL * lanes; ch < nchunk; ch += lanes) sum = cadd(sum, pw[c][int64_t(ch) * ncol]);
  }
  for (int off = lanes >> 1; off > 0; off >>= 1) {
    sum.x += __shfl_xor(sum.x, off);
    sum.y += __shfl_xor(sum.y, off);
  }
  if (!live || ln != 0) return;
  if (vert) sum = cadd(sum, cconv<C>(rv));
  rc[r * stride_c + gid] = cconv<Vout>(sum);
}

// rows[W][k]: owned fine rows of each wirebasket in footprint order; nrows[W] their count
__global__ void k_owned_rows(Geom g, const int* __restrict__ fpos, int nf,
                             const int* __restrict__ owner, int* __restrict__ rows,
                             int* __restrict__ nrows, int maxrows) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= g.nI * g.nJ) return;
  const int I = w / g.nJ, J = w - (w / g.nJ) * g.nJ;
  const int fpw = g.a + g.o;
  int k = 0;
  for (int fi = 0; fi < nf; ++fi) {
    const int pos = fpos[fi];
    const int dt = pos / fpw, dx = pos - (pos / fpw) * fpw;
    const int tt = g.a * I + dt, xx = g.a * J + dx;
    const int p = (tt >= g.Lt ? tt - g.Lt : tt) * g.Lx + (xx >= g.Lx ? xx - g.Lx : xx);
    if (owner[p] != w) continue;
    for (int i = 0; i < g.b && k < maxrows; ++i) rows[int64_t(w) * maxrows + k++] = p * g.b + i;
  }
  nrows[w] = k;
}

// Classification of every point: multiplicity 4 / 2 / 1 -> vertex / edge / interior.
__global__ void k_classify(Geom g, int8_t* __restrict__ kind, int* __restrict__ owner,
                           int* __restrict__ node) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.Lt * g.Lx) return;
  const int t = p / g.Lx, xc = p - (p / g.Lx) * g.Lx;
  const int It = t / g.a, Jx = xc / g.a;
  const bool two_t = (t % g.a) < g.o, two_x = (xc % g.a) < g.o;
  if (two_t && two_x) {
    kind[p] = 2;
    owner[p] = -1;
    node[p] = It * g.nJ + Jx;
    return;
  }
  node[p] = -1;
  if (two_t) {
    const int I2 = (It + g.nI - 1) % g.nI;
    kind[p] = 1;
    owner[p] = min(It, I2) * g.nJ + Jx;
  } else if (two_x) {
    const int J2 = (Jx + g.nJ - 1) % g.nJ;
    kind[p] = 1;
    owner[p] = It * g.nJ + min(Jx, J2);
  } else {
    kind[p] = 0;
    owner[p] = It * g.nJ + Jx;
  }
}

// splitmix64 first output (Steele, Lea, Flood 2014) of state s
__device__ inline uint64_t splitmix64(uint64_t s) {
  uint64_t z = s + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// W[k][dof] = u(re) + i u(im), u = (h >> 11) 2^-52 - 1, h = splitmix64(seed ^ key),
// key = (level << 56) | (k << 40) | (dof << 1) | part
__global__ void k_testvec_hash(uint64_t seed, int level, int nv, int64_t ndof, double2* W) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(nv) * ndof) return;
  const uint64_t k = uint64_t(i / ndof), dof = uint64_t(i % ndof);
  const uint64_t base = (uint64_t(level) << 56) | (k << 40) | (dof << 1);
  const uint64_t hre = splitmix64(seed ^ base), him = splitmix64(seed ^ (base | 1ull));
  W[i] = make_double2(double(hre >> 11) * 0x1p-52 - 1.0, double(him >> 11) * 0x1p-52 - 1.0);
}

// wc[k][N][(pt*o + px)*b + q] = w[k][vertex p][q]
__global__ void k_inject(Geom g, const int* __restrict__ node, const int8_t* __restrict__ kind,
                         const double2* __restrict__ w, double2* __restrict__ wc, int nv) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nd = g.ndof();
  if (i >= int64_t(nv) * nd) return;
  const int k = int(i / nd);
  const int64_t d = i - int64_t(k) * nd;
  const int p = int(d / g.b), q = int(d - int64_t(p) * g.b);
  if (kind[p] != 2) return;
  const int t = p / g.Lx, xc = p - (p / g.Lx) * g.Lx;
  const int pt = t % g.a, px = xc % g.a;
  const int64_t ncd = int64_t(g.nI) * g.nJ * g.bc;
  wc[int64_t(k) * ncd + int64_t(node[p]) * g.bc + (pt * g.o + px) * g.b + q] = w[i];
}

// ------------------------------------------------------------------------------ launchers

static size_t tile_smem(const TileShape& t, int ncol, int cs) {
  return size_t(t.rch) * (ncol + 1) * cs + size_t(t.rg) * (t.rch > ncol ? t.rch : ncol) * cs +
         size_t(t.rch) * sizeof(int);
}

// Pass 2 of the restriction.  CHL chunks per lane are loaded at once (the rest, if any, one
// after another); the sums run in the same order whatever CHL, so CHL only sets how many loads
// are in flight: as many as a lane has chunks, 1 or 2, else 8.
template <typename R, typename Vin, typename Vout>
static void launch_gather(hipStream_t s, dim3 g2, const void* part, const void* r, void* rc, const Geom& g,
                          int nchunk, int lanes, int64_t stride_f, int64_t stride_c, const RhsState* st) {
  if (nchunk > 2 * lanes)
    hipLaunchKernelGGL((k_restrict_gather<R, Vin, Vout, 8>), g2, dim3(256), 0, s, (const cplx<R>*)part,
                       (const Vin*)r, (Vout*)rc, g, nchunk, lanes, stride_f, stride_c, st);
  else if (nchunk <= lanes)
    hipLaunchKernelGGL((k_restrict_gather<R, Vin, Vout, 1>), g2, dim3(256), 0, s, (const cplx<R>*)part,
                       (const Vin*)r, (Vout*)rc, g, nchunk, lanes, stride_f, stride_c, st);
  else
    hipLaunchKernelGGL((k_restrict_gather<R, Vin, Vout, 2>), g2, dim3(256), 0, s, (const cplx<R>*)part,
                       (const Vin*)r, (Vout*)rc, g, nchunk, lanes, stride_f, stride_c, st);
}

int restrict_chunks(const Geom& g, int nf, Real prec) {
  if (prec == F32 && mfma_cols(g.ncol())) {
    return (nf * g.b + MfmaRows<128>::RESTRICT - 1) / MfmaRows<128>::RESTRICT;
  }
  if (tiled_cols(g.ncol())) {
    const int rch = prec == F64 ? TiledRows<double, 32>::RESTRICT : TiledRows<float, 32>::RESTRICT;
    return (nf * g.b + rch - 1) / rch;
  }
  return tile_shape(g.ncol(), prec == F64 ? 16 : 8, nf * g.b).nchunk;
}

template <int NCOL, typename R, typename M, typename V>
static void prolong_rows(hipStream_t s, const void* P, const int* rows, const int* nrows, int maxrows,
                         const void* e, void* y, const Geom& g, int add, int nrhs, int64_t stride_f,
                         int64_t stride_c, const RhsState* st) {
  const int nchunk = (maxrows + 63) / 64;
  AMAMG_LAUNCH((k_prolong_rows<NCOL, R, M, V, V>), dim3(unsigned(g.nI * g.nJ * nchunk)), dim3(64), 0, s,
               (const M*)P, rows, nrows, maxrows, (const V*)e, (V*)y, g, nchunk, add, nrhs, stride_f,
               stride_c, st);
}

template <int NCOL, typename R, typename M, typename V>
static void prolong_tiled(hipStream_t s, const void* P, const int* rows, const int* nrows, int maxrows,
                          const void* e, void* y, const Geom& g, int add, int nrhs, int64_t stride_f,
                          int64_t stride_c, const RhsState* st) {
  if (nrhs <= kRowsRhs) {
    prolong_rows<NCOL, R, M, V>(s, P, rows, nrows, maxrows, e, y, g, add, nrhs, stride_f, stride_c, st);
    return;
  }
  const int nchunk = (maxrows + TiledRows<R, NCOL>::PROLONG - 1) / TiledRows<R, NCOL>::PROLONG;
  AMAMG_LAUNCH((k_prolong_tiled<NCOL, TiledRows<R, NCOL>::PROLONG, TiledRows<R, NCOL>::RHS_P, R, M, V, V>), dim3(unsigned(g.nI * g.nJ * nchunk)), dim3(256), 0, s,
               (const M*)P, rows, nrows, maxrows, (const V*)e, (V*)y, g, nchunk, add, nrhs, stride_f,
               stride_c, st);
}

template <int NCOL>
static void prolong_mfma(hipStream_t s, const void* P, const int* rows, const int* nrows, int maxrows,
                         const void* e, void* y, const Geom& g, int add, int nrhs, int64_t stride_f,
                         int64_t stride_c, const RhsState* st) {
  if (nrhs <= 32) {
    constexpr int RCH32 = MfmaRows<NCOL>::PROLONG32;
    const int nchunk = (maxrows + RCH32 - 1) / RCH32;
    const dim3 grid(unsigned(g.nI * g.nJ * nchunk), 1);
    AMAMG_LAUNCH((k_prolong_mfma<NCOL, RCH32, 32>), grid, dim3(256), 0, s, (const float2*)P, rows, nrows, maxrows,
                 (const float2*)e, (float2*)y, g, nchunk, add, nrhs, stride_f, stride_c, st);
    return;
  }
  constexpr int RCH = MfmaRows<NCOL>::PROLONG;
  const int nchunk = (maxrows + RCH - 1) / RCH;
  const dim3 grid(unsigned(g.nI * g.nJ * nchunk), unsigned((nrhs + kMfmaRhs - 1) / kMfmaRhs));
  AMAMG_LAUNCH((k_prolong_mfma<NCOL, RCH, kMfmaRhs>), grid, dim3(256), 0, s, (const float2*)P, rows, nrows, maxrows,
               (const float2*)e, (float2*)y, g, nchunk, add, nrhs, stride_f, stride_c, st);
}

template <int NCOL, typename Vin>
static void restrict_mfma(hipStream_t s, const void* P, const int* rows, const int* nrows, int maxrows,
                          const void* r, void* part, int nW, int nchunk, int nrhs, int64_t stride_f,
                          const RhsState* st) {
  if (nrhs <= 32) {
    hipLaunchKernelGGL((k_restrict_mfma<NCOL, MfmaRows<NCOL>::RESTRICT, Vin, 32>), dim3(unsigned(nW * nchunk), 1),
                       dim3(256), 0, s, (const float2*)P, rows, nrows, maxrows, (const Vin*)r, (float2*)part, nW,
                       nchunk, nrhs, stride_f, st);
    return;
  }
  const dim3 grid(unsigned(nW * nchunk), unsigned((nrhs + kMfmaRhs - 1) / kMfmaRhs));
  hipLaunchKernelGGL((k_restrict_mfma<NCOL, MfmaRows<NCOL>::RESTRICT, Vin, kMfmaRhs>), grid, dim3(256), 0, s,
                     (const float2*)P, rows, nrows, maxrows, (const Vin*)r, (float2*)part, nW, nchunk, nrhs,
                     stride_f, st);
}

template <int NCOL, int RCH, typename R, typename M, typename Vin>
static void restrict_rows(hipStream_t s, const void* P, const int* rows, const int* nrows, int maxrows,
                          const void* r, void* part, int nW, int nchunk, int nrhs, int64_t stride_f,
                          const RhsState* st) {
  const dim3 grid(unsigned((nW * nchunk + kRowsChunks - 1) / kRowsChunks)), block(kRowsChunks * NCOL);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_restrict_rows<NCOL, RCH, 1, R, M, Vin>), grid, block, 0, s, (const M*)P, rows, nrows,
                       maxrows, (const Vin*)r, (cplx<R>*)part, nW, nchunk, nrhs, stride_f, st);
  else
    hipLaunchKernelGGL((k_restrict_rows<NCOL, RCH, kRowsRhs, R, M, Vin>), grid, block, 0, s, (const M*)P, rows,
                       nrows, maxrows, (const Vin*)r, (cplx<R>*)part, nW, nchunk, nrhs, stride_f, st);
}

template <int NCOL, typename R, typename M, typename Vin>
static void restrict_tiled(hipStream_t s, const void* P, const int* rows, const int* nrows, int maxrows,
                           const void* r, void* part, int nW, int nchunk, int nrhs, int64_t stride_f,
                           const RhsState* st) {
  if (nrhs <= kRowsRhs) {
    restrict_rows<NCOL, TiledRows<R, NCOL>::RESTRICT, R, M, Vin>(s, P, rows, nrows, maxrows, r, part, nW, nchunk,
                                                                nrhs, stride_f, st);
    return;
  }
  hipLaunchKernelGGL((k_restrict_partial_tiled<NCOL, TiledRows<R, NCOL>::RESTRICT, TiledRows<R, NCOL>::RHS_R, R, M, Vin>), dim3(unsigned(nW * nchunk)), dim3(256), 0,
                     s, (const M*)P, rows, nrows, maxrows, (const Vin*)r, (cplx<R>*)part, nW, nchunk, nrhs,
                     stride_f, st);
}

void owned_rows(hipStream_t s, const Geom& g, const int* fpos, int nf, const int* owner, int* rows,
                int* nrows) {
  hipLaunchKernelGGL(k_owned_rows, dim3((g.nI * g.nJ + 63) / 64), dim3(64), 0, s, g, fpos, nf, owner,
                     rows, nrows, nf * g.b);
}

void prolong(hipStream_t s, Real prec, const void* P, const int* rows, const int* nrows, int nf,
             const void* e, void* y, const Geom& g, int add, int nrhs, int64_t stride_f,
             int64_t stride_c, const RhsState* st) {
  const int cs = prec == F64 ? 16 : 8;
  const int maxrows = nf * g.b;
  if (prec == F32 && mfma_cols(g.ncol())) {
    prolong_mfma<128>(s, P, rows, nrows, maxrows, e, y, g, add, nrhs, stride_f, stride_c, st);
    return;
  }
  if (g.ncol() == 32) {
    if (prec == F64) prolong_tiled<32, double, double2, double2>(s, P, rows, nrows, maxrows, e, y, g, add, nrhs, stride_f, stride_c, st);
    else prolong_tiled<32, float, float2, float2>(s, P, rows, nrows, maxrows, e, y, g, add, nrhs, stride_f, stride_c, st);
    return;
  }
  if (g.ncol() == 8) {
    if (prec == F64) prolong_tiled<8, double, double2, double2>(s, P, rows, nrows, maxrows, e, y, g, add, nrhs, stride_f, stride_c, st);
    else prolong_tiled<8, float, float2, float2>(s, P, rows, nrows, maxrows, e, y, g, add, nrhs, stride_f, stride_c, st);
    return;
  }
  if (prec == F64 && g.bc == 32 && nrhs <= kRowsRhs) {
    const int nchunk = (maxrows + 63) / 64;
    AMAMG_LAUNCH((k_prolong_corner4<32, double, double2, double2, double2>), dim3(unsigned(g.nI * g.nJ * nchunk)),
                 dim3(256), 0, s, (const double2*)P, rows, nrows, maxrows, (const double2*)e, (double2*)y, g, nchunk,
                 add, nrhs, stride_f, stride_c, st);
    return;
  }
  const TileShape ts = tile_shape(g.ncol(), cs, nf * g.b);
  dim3 grid(unsigned(g.nI * g.nJ * ts.nchunk));
  const size_t sm = tile_smem(ts, g.ncol(), cs);
  if (prec == F64)
    AMAMG_LAUNCH((k_prolong<double, double2, double2, double2>), grid, dim3(256), sm, s,
                       (const double2*)P, rows, nrows, nf * g.b, (const double2*)e, (double2*)y, g,
                       ts, add, nrhs, stride_f, stride_c, st);
  else
    AMAMG_LAUNCH((k_prolong<float, float2, float2, float2>), grid, dim3(256), sm, s,
                       (const float2*)P, rows, nrows, nf * g.b, (const float2*)e, (float2*)y, g,
                       ts, add, nrhs, stride_f, stride_c, st);
}

void restrict_(hipStream_t s, Real prec, const void* P, const int* rows, const int* nrows, int nf,
               Real rin, const void* r, void* rc, void* part, const Geom& g, int nrhs,
               int64_t stride_f, int64_t stride_c, const RhsState* st) {
  const int cs = prec == F64 ? 16 : 8;
  const TileShape ts = tile_shape(g.ncol(), cs, nf * g.b);
  const int maxrows = nf * g.b;
  const int nchunk = restrict_chunks(g, nf, prec);
  int lanes = 1;
  while (lanes < 16 && lanes < nchunk) lanes <<= 1;
  dim3 g1(unsigned(g.nI * g.nJ * ts.nchunk));
  dim3 g2(unsigned((int64_t(g.nI) * g.nJ * g.bc * lanes + 255) / 256), unsigned(nrhs));
  const size_t sm = tile_smem(ts, g.ncol(), cs);
  const int nW = g.nI * g.nJ;
  if (prec == F32 && mfma_cols(g.ncol())) {
    if (rin == F64) restrict_mfma<128, double2>(s, P, rows, nrows, maxrows, r, part, nW, nchunk, nrhs, stride_f, st);
    else restrict_mfma<128, float2>(s, P, rows, nrows, maxrows, r, part, nW, nchunk, nrhs, stride_f, st);
    if (rin == F64)
      launch_gather<float, double2, float2>(s, g2, part, r, rc, g, nchunk, lanes, stride_f, stride_c, st);
    else
      launch_gather<float, float2, float2>(s, g2, part, r, rc, g, nchunk, lanes, stride_f, stride_c, st);
    return;
  }
  if (tiled_cols(g.ncol())) {
    if (g.ncol() == 32) {
      if (prec == F64) restrict_tiled<32, double, double2, double2>(s, P, rows, nrows, maxrows, r, part, nW, nchunk, nrhs, stride_f, st);
      else if (rin == F64) restrict_tiled<32, float, float2, double2>(s, P, rows, nrows, maxrows, r, part, nW, nchunk, nrhs, stride_f, st);
      else restrict_tiled<32, float, float2, float2>(s, P, rows, nrows, maxrows, r, part, nW, nchunk, nrhs, stride_f, st);
    } else {
      if (prec == F64) restrict_tiled<8, double, double2, double2>(s, P, rows, nrows, maxrows, r, part, nW, nchunk, nrhs, stride_f, st);
      else if (rin == F64) restrict_tiled<8, float, float2, double2>(s, P, rows, nrows, maxrows, r, part, nW, nchunk, nrhs, stride_f, st);
      else restrict_tiled<8, float, float2, float2>(s, P, rows, nrows, maxrows, r, part, nW, nchunk, nrhs, stride_f, st);
    }
    if (prec == F64)
      launch_gather<double, double2, double2>(s, g2, part, r, rc, g, nchunk, lanes, stride_f, stride_c, st);
    else if (rin == F64)
      launch_gather<float, double2, float2>(s, g2, part, r, rc, g, nchunk, lanes, stride_f, stride_c, st);
    else
      launch_gather<float, float2, float2>(s, g2, part, r, rc, g, nchunk, lanes, stride_f, stride_c, st);
    return;
  }
  if (prec == F64) {
    // level 1 of a = 8, o = 2: 128 columns in chunks of 8 rows
    if (g.ncol() == 128 && ts.rch == 8 && nrhs <= kRowsRhs)
      restrict_rows<128, 8, double, double2, double2>(s, P, rows, nrows, maxrows, r, part, nW, ts.nchunk, nrhs,
                                                      stride_f, st);
    else
      hipLaunchKernelGGL((k_restrict_partial<double, double2, double2>), g1, dim3(256), sm, s,
                         (const double2*)P, rows, nrows, maxrows, (const double2*)r, (double2*)part, g,
                         ts, nrhs, stride_f, st);
    launch_gather<double, double2, double2>(s, g2, part, r, rc, g, ts.nchunk, lanes, stride_f, stride_c, st);
  } else if (rin == F64) {
    hipLaunchKernelGGL((k_restrict_partial<float, float2, double2>), g1, dim3(256), sm, s,
                       (const float2*)P, rows, nrows, maxrows, (const double2*)r, (float2*)part, g,
                       ts, nrhs, stride_f, st);
    launch_gather<float, double2, float2>(s, g2, part, r, rc, g, ts.nchunk, lanes, stride_f, stride_c, st);
  } else {
    hipLaunchKernelGGL((k_restrict_partial<float, float2, float2>), g1, dim3(256), sm, s,
                       (const float2*)P, rows, nrows, maxrows, (const float2*)r, (float2*)part, g,
                       ts, nrhs, stride_f, st);
    launch_gather<float, float2, float2>(s, g2, part, r, rc, g, ts.nchunk, lanes, stride_f, stride_c, st);
  }
}

void classify(hipStream_t s, const Geom& g, int8_t* kind, int* owner, int* node) {
  hipLaunchKernelGGL(k_classify, dim3((g.Lt * g.Lx + 255) / 256), dim3(256), 0, s, g, kind, owner,
                     node);
}

void testvec_hash(hipStream_t s, uint64_t seed, int level, int nv, int64_t ndof, double2* W) {
  const int64_t n = int64_t(nv) * ndof;
  hipLaunchKernelGGL(k_testvec_hash, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, seed, level,
                     nv, ndof, W);
}

void inject(hipStream_t s, const Geom& g, const int* node, const int8_t* kind, const double2* w,
            double2* wc, int nv) {
  const int64_t n = int64_t(nv) * g.ndof();
  hipLaunchKernelGGL(k_inject, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, g, node, kind, w,
                     wc, nv);
}

}  // namespace amamg
