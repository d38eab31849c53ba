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
#include "launch.hpp"

namespace amamg {

__device__ inline int wrap_s(int v, int L) { v %= L; return v < 0 ? v + L : v; }

// Aff [W][nfd][nfd], Bneg [W][nfd][ncol]; A: block stencil [node][noff][b][b]
__global__ __launch_bounds__(256) void k_gather_local(Geom g, const double2* __restrict__ A, int noff,
                                                      const int* __restrict__ offs,
                                                      const int* __restrict__ postab,
                                                      const int* __restrict__ fpos, int nf,
                                                      double2* __restrict__ Aff,
                                                      double2* __restrict__ Bneg) {
  const int w = blockIdx.x;
  const int I = w / g.nJ, J = w - (w / g.nJ) * g.nJ;
  const int fpw = g.a + g.o;
  const int nfd = nf * g.b, ncol = g.ncol();
  double2* Aw = Aff + int64_t(w) * nfd * nfd;
  double2* Bw = Bneg + int64_t(w) * nfd * ncol;
  for (int64_t e = threadIdx.x; e < int64_t(nfd) * nfd; e += blockDim.x) Aw[e] = make_double2(0, 0);
  for (int64_t e = threadIdx.x; e < int64_t(nfd) * ncol; e += blockDim.x) Bw[e] = make_double2(0, 0);
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
        double2* dst = Aw + int64_t(rrow) * nfd + int64_t(code) * g.b;
        for (int j = 0; j < g.b; ++j) dst[j] = cadd(dst[j], blk[j]);
      } else {
        double2* dst = Bw + int64_t(rrow) * ncol + (-code - 1);
        for (int j = 0; j < g.b; ++j) dst[j] = csub(dst[j], blk[j]);
      }
    }
  }
}

// In-place LU with partial pivoting (largest |a_ik|, lowest index on ties) of one n x n
// row-major system per workgroup.  info[sys] = 0, or k + 1 for a zero pivot at step k.
__global__ __launch_bounds__(256) void k_lu_factor(double2* __restrict__ A, int n, int* __restrict__ piv,
                                                   int* __restrict__ info) {
  const int sys = blockIdx.x;
  double2* M = A + int64_t(sys) * n * n;
  int* pv = piv + int64_t(sys) * n;
  __shared__ double sv[256];
  __shared__ int si[256];
  const int tid = threadIdx.x;
  if (tid == 0) info[sys] = 0;
  for (int k = 0; k < n; ++k) {
    double best = -1.0;
    int bi = n;
    for (int i = k + tid; i < n; i += 256) {
      const double v = cabs2(M[int64_t(i) * n + k]);
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
    if (!(pmax > 0.0) || p >= n) {       // zero or non-finite pivot column
      if (tid == 0) info[sys] = k + 1;
      for (int kk = k + tid; kk < n; kk += 256) pv[kk] = kk;
      return;
    }
    if (tid == 0) pv[k] = p;
    if (p != k) {
      for (int j = tid; j < n; j += 256) {
        const double2 t = M[int64_t(k) * n + j];
        M[int64_t(k) * n + j] = M[int64_t(p) * n + j];
        M[int64_t(p) * n + j] = t;
      }
    }
    __syncthreads();
    const double2 akk = M[int64_t(k) * n + k];
    const double den = cabs2(akk);
    const double2 inv = make_double2(akk.x / den, -akk.y / den);
    for (int i = k + 1 + tid; i < n; i += 256) M[int64_t(i) * n + k] = cmul(M[int64_t(i) * n + k], inv);
    __syncthreads();
    // trailing update: wave wv takes rows k+1+wv, k+5+wv, ...; lanes sweep the columns
    const int lane = tid & 63, wv = tid >> 6;
    for (int i = k + 1 + wv; i < n; i += 4) {
      const double2 lik = M[int64_t(i) * n + k];
      double2* Mi = M + int64_t(i) * n;
      const double2* Mk = M + int64_t(k) * n;
      for (int j = k + 1 + lane; j < n; j += 64) Mi[j] = csub(Mi[j], cmul(lik, Mk[j]));
    }
    __syncthreads();
  }
}

// Solve with the factors for nrhs right-hand sides B [sys][n][nrhs]; one thread per column.
__global__ __launch_bounds__(64) void k_lu_solve(const double2* __restrict__ LU, const int* __restrict__ piv,
                                                 int n, double2* __restrict__ B, int nrhs) {
  const int sys = blockIdx.x;
  const int col = blockIdx.y * 64 + threadIdx.x;
  if (col >= nrhs) return;
  const double2* M = LU + int64_t(sys) * n * n;
  const int* pv = piv + int64_t(sys) * n;
  double2* Bs = B + int64_t(sys) * n * nrhs + col;
  for (int k = 0; k < n; ++k) {
    const int p = pv[k];
    if (p != k) {
      const double2 t = Bs[int64_t(k) * nrhs];
      Bs[int64_t(k) * nrhs] = Bs[int64_t(p) * nrhs];
      Bs[int64_t(p) * nrhs] = t;
    }
  }
  for (int i = 1; i < n; ++i) {
    double2 acc = Bs[int64_t(i) * nrhs];
    for (int k = 0; k < i; ++k) acc = csub(acc, cmul(M[int64_t(i) * n + k], Bs[int64_t(k) * nrhs]));
    Bs[int64_t(i) * nrhs] = acc;
  }
  for (int i = n - 1; i >= 0; --i) {
    double2 acc = Bs[int64_t(i) * nrhs];
    for (int k = i + 1; k < n; ++k) acc = csub(acc, cmul(M[int64_t(i) * n + k], Bs[int64_t(k) * nrhs]));
    const double2 d = M[int64_t(i) * n + i];
    const double den = cabs2(d);
    Bs[int64_t(i) * nrhs] = cmul(acc, make_double2(d.x / den, -d.y / den));
  }
}

// Copy the rows of each wirebasket's solution that the wirebasket owns into P [p][i][ncol].
__global__ void k_scatter_P(Geom g, const double2* __restrict__ X, const int* __restrict__ fpos,
                            int nf, const int* __restrict__ owner, double2* __restrict__ P) {
  const int w = blockIdx.x;
  const int I = w / g.nJ, J = w - (w / g.nJ) * g.nJ;
  const int fpw = g.a + g.o, ncol = g.ncol(), nfd = nf * g.b;
  const double2* Xw = X + int64_t(w) * nfd * ncol;
  for (int64_t e = threadIdx.x; e < int64_t(nfd) * ncol; e += blockDim.x) {
    const int rrow = int(e / ncol), col = int(e - int64_t(rrow) * ncol);
    const int fi = rrow / g.b, i = rrow - (rrow / g.b) * g.b;
    const int pos = fpos[fi];
    const int dt = pos / fpw, dx = pos - (pos / fpw) * fpw;
    const int p = wrap_s(g.a * I + dt, g.Lt) * g.Lx + wrap_s(g.a * J + dx, g.Lx);
    if (owner[p] != w) continue;
    P[(int64_t(p) * g.b + i) * ncol + col] = Xw[e];
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

__global__ void k_extract_diag(const double2* __restrict__ A, int nnode, int b, double2* __restrict__ D) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(nnode) * b * b) return;
  const int64_t n = i / (b * b), e = i - n * b * b;
  D[i] = A[(n * 25 + 12) * b * b + e];
}

__global__ void k_set_identity(double2* __restrict__ B, int n, int nsys) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(nsys) * n * n) return;
  const int64_t e = i % (int64_t(n) * n);
  const int r = int(e / n), c = int(e - int64_t(r) * n);
  B[i] = make_double2(r == c ? 1.0 : 0.0, 0.0);
}

__global__ void k_cast_matrix(const double2* __restrict__ A, float2* __restrict__ out, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2(float(A[i].x), float(A[i].y));
}

// ------------------------------------------------------------------------------ launchers

static inline dim3 g1(int64_t n) { return dim3(unsigned((n + 255) / 256)); }

void gather_local(hipStream_t s, const Geom& g, const double2* A, int noff, const int* offs,
                  const int* postab_fpos, int nf, double2* Aff, double2* Bneg) {
  const int fp = g.fp();
  hipLaunchKernelGGL(k_gather_local, dim3(g.nI * g.nJ), dim3(256), 0, s, g, A, noff, offs,
                     postab_fpos, postab_fpos + fp, nf, Aff, Bneg);
}

void lu_factor(hipStream_t s, double2* A, int n, int nsys, int* piv, int* info) {
  hipLaunchKernelGGL(k_lu_factor, dim3(nsys), dim3(256), 0, s, A, n, piv, info);
}

void lu_solve(hipStream_t s, const double2* LU, const int* piv, int n, int nsys, double2* B,
              int nrhs) {
  hipLaunchKernelGGL(k_lu_solve, dim3(nsys, (nrhs + 63) / 64), dim3(64), 0, s, LU, piv, n, B, nrhs);
}

void scatter_P(hipStream_t s, const Geom& g, const double2* X, const int* postab_fpos, int nf,
               const int* owner, double2* P) {
  hipLaunchKernelGGL(k_scatter_P, dim3(g.nI * g.nJ), dim3(256), 0, s, g, X, postab_fpos + g.fp(),
                     nf, owner, P);
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

void extract_diag(hipStream_t s, const double2* A, int nnode, int b, double2* D) {
  hipLaunchKernelGGL(k_extract_diag, g1(int64_t(nnode) * b * b), dim3(256), 0, s, A, nnode, b, D);
}

void set_identity(hipStream_t s, double2* B, int n, int nsys) {
  hipLaunchKernelGGL(k_set_identity, g1(int64_t(nsys) * n * n), dim3(256), 0, s, B, n, nsys);
}

void cast_matrix(hipStream_t s, const double2* A, float2* out, int64_t n) {
  hipLaunchKernelGGL(k_cast_matrix, g1(n), dim3(256), 0, s, A, out, n);
}

}  // namespace amamg
