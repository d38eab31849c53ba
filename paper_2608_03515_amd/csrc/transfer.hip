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
// node ((I+ct) mod nI, (J+cx) mod nJ) of p's primary wirebasket, bc = o*o*b.  Vertex rows are
// the identity and are not stored (left zero).
#include "launch.hpp"

namespace amamg {

__device__ inline int wrapt(int v, int L) { v %= L; return v < 0 ? v + L : v; }

__device__ inline int corner_node(int w, int c, int nI, int nJ) {
  const int I = w / nJ, J = w - (w / nJ) * nJ;
  const int ct = c >> 1, cx = c & 1;
  return ((I + ct) % nI) * nJ + (J + cx) % nJ;
}

__device__ inline int lanes_per_row(int ncol) {
  int g = 1;
  while (g < 32 && g < ncol) g <<= 1;
  return g;
}

// y[p][i] = sum_col P[p][i][col] e[corner(col)][col mod bc]  (F rows)
// y[p][i] = e[node(p)][(pt*o + px)*b + i]                  (vertex rows)
// G lanes share a row (strided columns, then a shuffle reduction); 64/G rows per wave.
template <typename R, typename M, typename Vin, typename Vout>
__global__ __launch_bounds__(256) void k_prolong(const M* __restrict__ P,
                                                 const int* __restrict__ owner,
                                                 const int* __restrict__ node,
                                                 const Vin* __restrict__ e,
                                                 Vout* __restrict__ y, Geom g, int add,
                                                 int64_t stride_f, int64_t stride_c,
                                                 const RhsState* __restrict__ st) {
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  using C = cplx<R>;
  const int ncol = g.ncol();
  const int G = lanes_per_row(ncol);
  const int rows_per_block = 256 / G;
  const int lane_g = threadIdx.x % G;
  const int64_t row = int64_t(xcd_block(blockIdx.x, gridDim.x)) * rows_per_block + threadIdx.x / G;
  const int64_t nrow = g.ndof();
  const bool live = row < nrow;
  const int p = live ? int(row / g.b) : 0;
  const int i = live ? int(row - int64_t(p) * g.b) : 0;
  const Vin* er = e + r * stride_c;
  C acc = czero<R>();
  const int w = live ? owner[p] : -1;
  if (w >= 0) {
    const M* Pr = P + row * ncol;
    for (int col = lane_g; col < ncol; col += G) {
      const int c = col / g.bc, j = col - c * g.bc;
      const int cn = corner_node(w, c, g.nI, g.nJ);
      acc = cfma(cconv<C>(Pr[col]), cconv<C>(er[int64_t(cn) * g.bc + j]), acc);
    }
  }
  // reduce over the G lanes of this row (aligned groups, so xor stays inside the group)
  for (int off = G >> 1; off > 0; off >>= 1) {
    acc.x += __shfl_xor(acc.x, off);
    acc.y += __shfl_xor(acc.y, off);
  }
  if (live && lane_g == 0) {
    if (w < 0) {
      const int t = p / g.Lx, xc = p - (p / g.Lx) * g.Lx;
      const int pt = t % g.a, px = xc % g.a;
      acc = cconv<C>(er[int64_t(node[p]) * g.bc + (pt * g.o + px) * g.b + i]);
    }
    Vout* yr = y + r * stride_f;
    if (add) acc = cadd(acc, cconv<C>(yr[row]));
    yr[row] = cconv<Vout>(acc);
  }
}

// Restriction rc = P^H r in two passes, both fixed-order (deterministic, no atomics).
// Pass 1, one workgroup per (wirebasket W, chunk of W's owned rows): for every interpolation
// column col of W, part[W][chunk][col] = sum over the chunk's rows of conj(P[row][col]) r[row].
// rows[W][k] lists W's owned fine rows (p*b + i) in footprint order (nrows[W] of them); the
// chunk's r values are staged in LDS, lanes run over columns, so each P row is read as one
// contiguous segment.
// Pass 2: rc[N][j] = sum over the 4 wirebaskets W having N as corner c and over their chunks
// of part[W][chunk][c*bc + j], plus r at N's vertices; L lanes per output, xor-reduced.
#define RCHUNK_MAX 256
template <typename R, typename M, typename Vin>
__global__ __launch_bounds__(256) void k_restrict_partial(const M* __restrict__ P,
                                                          const int* __restrict__ rows,
                                                          const int* __restrict__ nrows,
                                                          int maxrows,
                                                          const Vin* __restrict__ rin,
                                                          cplx<R>* __restrict__ part, Geom g,
                                                          int nchunk, int64_t stride_f,
                                                          const RhsState* __restrict__ st) {
  const int r = blockIdx.y;
  if (st && !st[r].active) return;
  using C = cplx<R>;
  __shared__ R red[2][256];
  __shared__ C rs[RCHUNK_MAX];
  __shared__ int ri[RCHUNK_MAX];
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int w = bid / nchunk, chunk = bid - (bid / nchunk) * nchunk;
  const int ncol = g.ncol();
  const int nr = nrows[w];
  const int rpc = (maxrows + nchunk - 1) / nchunk;
  const int r0 = chunk * rpc, r1 = min(nr, r0 + rpc);
  const int cnt = r1 > r0 ? r1 - r0 : 0;
  const Vin* rr = rin + r * stride_f;
  for (int k = threadIdx.x; k < cnt; k += 256) {
    const int row = rows[int64_t(w) * maxrows + r0 + k];
    ri[k] = row;
    rs[k] = cconv<C>(rr[row]);
  }
  __syncthreads();
  const int CW = ncol < 256 ? ncol : 256;
  const int nslot = 256 / CW;
  const int cl = threadIdx.x % CW, slot = threadIdx.x / CW;
  C* out = part + ((int64_t(r) * g.nI * g.nJ + w) * nchunk + chunk) * ncol;
  for (int c0 = 0; c0 < ncol; c0 += CW) {
    const int col = c0 + cl;
    C acc = czero<R>();
    if (slot < nslot && col < ncol) {
      int k = slot;
      for (; k + 3 * nslot < cnt; k += 4 * nslot) {
        const M p0 = P[int64_t(ri[k]) * ncol + col];
        const M p1 = P[int64_t(ri[k + nslot]) * ncol + col];
        const M p2 = P[int64_t(ri[k + 2 * nslot]) * ncol + col];
        const M p3 = P[int64_t(ri[k + 3 * nslot]) * ncol + col];
        acc = cfmac(cconv<C>(p0), rs[k], acc);
        acc = cfmac(cconv<C>(p1), rs[k + nslot], acc);
        acc = cfmac(cconv<C>(p2), rs[k + 2 * nslot], acc);
        acc = cfmac(cconv<C>(p3), rs[k + 3 * nslot], acc);
      }
      for (; k < cnt; k += nslot) acc = cfmac(cconv<C>(P[int64_t(ri[k]) * ncol + col]), rs[k], acc);
    }
    red[0][threadIdx.x] = acc.x;
    red[1][threadIdx.x] = acc.y;
    __syncthreads();
    if (slot == 0 && col < ncol) {
      C sum = czero<R>();
      for (int q = 0; q < nslot; ++q) sum = cadd(sum, mk<R>(red[0][q * CW + cl], red[1][q * CW + cl]));
      out[col] = sum;
    }
    __syncthreads();
  }
}

template <typename R, typename Vin, typename Vout>
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
  C sum = czero<R>();
  for (int c = 0; c < 4; ++c) {
    const int WI = I - (c >> 1), WJ = J - (c & 1);
    const int w = (WI < 0 ? WI + g.nI : WI) * g.nJ + (WJ < 0 ? WJ + g.nJ : WJ);
    const C* pw = part + (int64_t(r) * nW + w) * nchunk * ncol + c * g.bc + j;
    for (int ch = ln; ch < nchunk; ch += lanes) sum = cadd(sum, pw[int64_t(ch) * ncol]);
  }
  for (int off = lanes >> 1; off > 0; off >>= 1) {
    sum.x += __shfl_xor(sum.x, off);
    sum.y += __shfl_xor(sum.y, off);
  }
  if (!live || ln != 0) return;
  const int q = j % g.b, pp = j / g.b;
  const int pt = pp / g.o, px = pp - (pp / g.o) * g.o;
  const int p = (g.a * I + pt) * g.Lx + (g.a * J + px);
  sum = cadd(sum, cconv<C>(rin[r * stride_f + int64_t(p) * g.b + q]));
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

void prolong(hipStream_t s, Real prec, const void* P, const int* owner, const int* node,
             const void* e, void* y, const Geom& g, int add, int nrhs, int64_t stride_f,
             int64_t stride_c, const RhsState* st) {
  int G = 1;
  while (G < 32 && G < g.ncol()) G <<= 1;
  const int rows_per_block = 256 / G;
  dim3 grid(unsigned((g.ndof() + rows_per_block - 1) / rows_per_block), unsigned(nrhs));
  if (prec == F64)
    hipLaunchKernelGGL((k_prolong<double, double2, double2, double2>), grid, dim3(256), 0, s,
                       (const double2*)P, owner, node, (const double2*)e, (double2*)y, g, add,
                       stride_f, stride_c, st);
  else
    hipLaunchKernelGGL((k_prolong<float, float2, float2, float2>), grid, dim3(256), 0, s,
                       (const float2*)P, owner, node, (const float2*)e, (float2*)y, g, add,
                       stride_f, stride_c, st);
}

int restrict_chunks(const Geom& g, int nf) {
  const int nW = g.nI * g.nJ, nfd = nf * g.b;
  int nchunk = (1024 + nW - 1) / nW;
  const int maxc = (nfd + 7) / 8;
  if (nchunk > maxc) nchunk = maxc;
  while ((nfd + nchunk - 1) / nchunk > RCHUNK_MAX) ++nchunk;
  return nchunk < 1 ? 1 : nchunk;
}

void owned_rows(hipStream_t s, const Geom& g, const int* fpos, int nf, const int* owner, int* rows,
                int* nrows) {
  hipLaunchKernelGGL(k_owned_rows, dim3((g.nI * g.nJ + 63) / 64), dim3(64), 0, s, g, fpos, nf, owner,
                     rows, nrows, nf * g.b);
}

void restrict_(hipStream_t s, Real prec, const void* P, const int* rows, const int* nrows, int nf,
               Real rin, const void* r, void* rc, void* part, const Geom& g, int nrhs,
               int64_t stride_f, int64_t stride_c, const RhsState* st) {
  const int nchunk = restrict_chunks(g, nf);
  const int maxrows = nf * g.b;
  int lanes = 1;
  while (lanes < 16 && lanes < nchunk) lanes <<= 1;
  dim3 g1(unsigned(g.nI * g.nJ * nchunk), unsigned(nrhs));
  dim3 g2(unsigned((int64_t(g.nI) * g.nJ * g.bc * lanes + 255) / 256), unsigned(nrhs));
  if (prec == F64) {
    hipLaunchKernelGGL((k_restrict_partial<double, double2, double2>), g1, dim3(256), 0, s,
                       (const double2*)P, rows, nrows, maxrows, (const double2*)r, (double2*)part, g,
                       nchunk, stride_f, st);
    hipLaunchKernelGGL((k_restrict_gather<double, double2, double2>), g2, dim3(256), 0, s,
                       (const double2*)part, (const double2*)r, (double2*)rc, g, nchunk, lanes,
                       stride_f, stride_c, st);
  } else if (rin == F64) {
    hipLaunchKernelGGL((k_restrict_partial<float, float2, double2>), g1, dim3(256), 0, s,
                       (const float2*)P, rows, nrows, maxrows, (const double2*)r, (float2*)part, g,
                       nchunk, stride_f, st);
    hipLaunchKernelGGL((k_restrict_gather<float, double2, float2>), g2, dim3(256), 0, s,
                       (const float2*)part, (const double2*)r, (float2*)rc, g, nchunk, lanes,
                       stride_f, stride_c, st);
  } else {
    hipLaunchKernelGGL((k_restrict_partial<float, float2, float2>), g1, dim3(256), 0, s,
                       (const float2*)P, rows, nrows, maxrows, (const float2*)r, (float2*)part, g,
                       nchunk, stride_f, st);
    hipLaunchKernelGGL((k_restrict_gather<float, float2, float2>), g2, dim3(256), 0, s,
                       (const float2*)part, (const float2*)r, (float2*)rc, g, nchunk, lanes,
                       stride_f, stride_c, st);
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
