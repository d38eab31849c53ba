// Host-side launchers of the HIP kernels (one declaration per operation; the definitions sit
// beside their kernels).  All launches are asynchronous on `s`.
#pragma once

#include <hip/hip_ext.h>

#include "common.hpp"

namespace amamg {

// Kernel-timer hook (host side, per thread).  When `start` is set, the next launch through
// AMAMG_LAUNCH stamps `start` and `stop` at that kernel's own begin and end (the times a kernel
// trace reports, without the queueing a pair of stream events would also measure) and clears
// the hook.
struct TimedLaunch {
  hipEvent_t start = nullptr, stop = nullptr;
};
TimedLaunch& timed_launch();

#define AMAMG_LAUNCH(kernel, grid, block, shmem, stream, ...)                                   \
  do {                                                                                          \
    ::amamg::TimedLaunch& tl_ = ::amamg::timed_launch();                                        \
    if (tl_.start) {                                                                            \
      const ::amamg::TimedLaunch ev_ = tl_;                                                     \
      tl_ = ::amamg::TimedLaunch{};                                                             \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, ev_.start, ev_.stop, 0, __VA_ARGS__); \
    } else {                                                                                    \
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                      \
    }                                                                                           \
  } while (0)

enum Real { F64 = 0, F32 = 1 };
enum LinkStore { LINK_F64 = 0, LINK_F32 = 1, LINK_BF16 = 2 };

// Geometry of one level's grid and of its wirebaskets (for the transfer to the next level).
struct Geom {
  int Lt, Lx, b;      // grid and degrees of freedom per node
  int a, o;           // aggregate size, overlap
  int nI, nJ;         // wirebaskets per direction (Lt / a, Lx / a)
  int bv;             // vertex degrees of freedom per coarse node (o * o * b)
  int bc;             // degrees of freedom per coarse node: bv, plus the augmented ones
  __host__ __device__ int nnode() const { return Lt * Lx; }
  __host__ __device__ int64_t ndof() const { return int64_t(Lt) * Lx * b; }
  __host__ __device__ int ncol() const { return 4 * bc; }   // interpolation columns per row
  __host__ __device__ int nvcol() const { return 4 * bv; }  // columns of the local systems' V part
  __host__ __device__ int fp() const { return (a + o) * (a + o); }
};

// ---- fine level (Wilson stencil); vectors [rhs][site][2 spin] complex ---------------------
// y = D x   (x: vin; y: vout; b == nullptr)  or  y = b - D x  (b: FP64 right-hand side)
void wilson_apply(hipStream_t s, LinkStore ls, const void* U0, const void* U1, Real vin,
                  const void* x, Real vout, void* y, const double2* b, int nt, int nx, double m0,
                  int nrhs, int64_t stride, const RhsState* st);
// one colour of the red-black point Gauss-Seidel sweep on D x = b (b FP64 or null = 0)
void wilson_gs(hipStream_t s, LinkStore ls, const void* U0, const void* U1, Real vx, void* x,
               const double2* b, int nt, int nx, double m0, int colour, int nrhs, int64_t stride,
               const RhsState* st);
// `sweeps` (1 or 2) full red-black sweeps (colour 0 then 1 each) in one launch, starting from xin
// and writing x (distinct buffers); bitwise equal to the same sequence of wilson_gs colour
// launches on x = xin.  tc = tile width in sites (16, 32, 64 FP32; 16, 32 FP64; 0 = default):
// a launch parameter only, the results do not depend on it
void wilson_gs_sweeps(hipStream_t s, LinkStore ls, const void* U0, const void* U1, Real vx, const void* xin,
                      void* x, const double2* b, int nt, int nx, double m0, int sweeps, int nrhs,
                      int64_t stride, const RhsState* st, int tc = 0);
// A0 blocks of the fine operator in block-stencil form: [site][5][2][2], offsets
// (0,0), (+1,0), (-1,0), (0,+1), (0,-1)
void build_fine_stencil(hipStream_t s, const double2* U0, const double2* U1, int nt, int nx,
                        double m0, double2* A0);
// link copies in lower precision (FP32, BF16 round to nearest even)
void links_to_f32(hipStream_t s, const double2* U, float2* out, int64_t n);
void links_to_bf16(hipStream_t s, const double2* U, bf16c* out, int64_t n);
// canonical <-> internal is the identity; casts between vector precisions
void cast_vec(hipStream_t s, Real from, const void* x, Real to, void* y, int64_t n);

// ---- coarse levels (block stencil [node][25][b][b]) -------------------------------------
// y = A x or y = f - A x (f non-null, same type as vout)
void stencil_apply(hipStream_t s, Real prec, const void* A, const void* x, void* y,
                   const void* f, int Lt, int Lx, int b, int nrhs, int64_t stride,
                   const RhsState* st);
// one colour of the 16-colour point-block Gauss-Seidel sweep: x_n = Dinv_n (f_n - sum_{d!=0} A_nd x_{n+d})
// f may be null (zero right-hand side)
void stencil_gs(hipStream_t s, Real prec, const void* A, const void* Dinv, void* x, const void* f,
                int Lt, int Lx, int b, int colour, int nrhs, int64_t stride, const RhsState* st);
// FP32 8 x 8 block sweeps run on matrix cores (mode 1), on the vector kernels (mode 2) or, by
// default (mode 0), on matrix cores from 32 x 32 nodes up (enough 2 x 2 groups per launch).
// Fixed per hierarchy level, so a right-hand side's result never depends on its batch.
inline bool gs_on_matrix_cores(int Lt, int Lx, int mode) {
  return mode == 1 || (mode == 0 && Lt * Lx >= 1024);
}
constexpr int kGsNodeWaves = -4;
// colour block qb (0..3) of the coarse sweep order (coarse_colour(4 qb) .. coarse_colour(4 qb +
// 3)).  FP32 8 x 8 blocks with gs_on_matrix_cores(mode): one matrix-core launch, variant = offsets
// per load batch (8, 12 or 24; 0 = 12).  Otherwise bitwise equal to four stencil_gs launches
// in that order; variant (FP32 8 x 8 blocks): > 0 colour-pair launches with that many
// right-hand sides per wave, -1 and -2 one launch per block with -variant right-hand sides per
// wave, kGsNodeWaves one launch per block with one wave per node and one right-hand side per
// workgroup.  The variant is a launch parameter only
void stencil_gs_block(hipStream_t s, Real prec, const void* A, const void* Dinv, void* x, const void* f,
                      int Lt, int Lx, int b, int qb, int nrhs, int64_t stride, const RhsState* st, int variant = 0,
                      int mode = 0);
// coarsest, GMRES variant: x = unpreconditioned GMRES(A, f) from 0 to relative tolerance tol in
// at most `steps` (<= 32) steps, n <= 2048; Acm column-major FP64; basis [nrhs][steps + 1][n]
void coarsest_gmres(hipStream_t s, Real prec, const double2* Acm, const void* f, void* x, int n, int nrhs,
                    int64_t stride, const RhsState* st, double tol, int steps, double2* basis);
void transpose_dense(hipStream_t s, const double2* A, double2* At, int n);
constexpr int kCoarsestGmresMaxSteps = 32, kCoarsestGmresMaxN = 2048;
// coarsest: y = Ainv v (matrix FP64 always; vectors in prec)
void dense_apply(hipStream_t s, Real prec, const double2* Ainv, const void* v, void* y, int n,
                 int nrhs, int64_t stride, const RhsState* st);

// ---- transfer between level k (fine side, geometry g) and k+1 ----------------------------
// rows/nrows: the owned fine rows of each wirebasket in footprint order (owned_rows).
void owned_rows(hipStream_t s, const Geom& g, const int* fpos, int nf, const int* owner, int* rows,
                int* nrows);
// y = P e   (add != 0: y += P e); e: coarse vectors in prec; y: fine vectors in prec
void prolong(hipStream_t s, Real prec, const void* P, const int* rows, const int* nrows, int nf,
             const void* e, void* y, const Geom& g, int add, int nrhs, int64_t stride_f,
             int64_t stride_c, const RhsState* st);
// rc = P^H r; r in `rin` precision (FP64 basis vector or prec), rc in prec; part: scratch of
// nrhs * nW * restrict_chunks(g, nf, prec) * ncol complex values in prec.
int restrict_chunks(const Geom& g, int nf, Real prec);
void restrict_(hipStream_t s, Real prec, const void* P, const int* rows, const int* nrows, int nf,
               Real rin, const void* r, void* rc, void* part, const Geom& g, int nrhs,
               int64_t stride_f, int64_t stride_c, const RhsState* st);

// ---- setup -------------------------------------------------------------------------------
void classify(hipStream_t s, const Geom& g, int8_t* kind, int* owner, int* node);
void testvec_hash(hipStream_t s, uint64_t seed, int level, int nv, int64_t ndof, double2* W);
void inject(hipStream_t s, const Geom& g, const int* node, const int8_t* kind, const double2* w,
            double2* wc, int nv);
// local systems of every wirebasket: Aug [W][nfd][nfd + ncol] = [A_FF | -A_FV]
void gather_local(hipStream_t s, const Geom& g, const double2* A, int noff, const int* offs_dev,
                  const int* postab, int nf, double2* Aug);
// batched dense solves on augmented [A | B] (n x (n + nrhs) row-major per system): B <- A^-1 B;
// info: nsys * kDenseSolveInts ints, info[sys] = 0 or the first zero pivot column + 1 (the
// rest is the solver's scratch)
constexpr int kDenseSolveInts = 17;
void dense_solve(hipStream_t s, double2* Aug, int n, int nrhs, int nsys, int* info);
void aug_extract(hipStream_t s, const double2* Aug, int n, int nrhs, double2* out, int nsys);
// Aug = [A | I] from nsys n x n blocks at stride astride with row stride arow
void aug_identity(hipStream_t s, const double2* A, int64_t astride, int arow, int n, double2* Aug,
                  int nsys);
void scatter_P(hipStream_t s, const Geom& g, const double2* X, const int* postab, int nf,
               const int* owner, double2* P);
// augmented coarse space: per wirebasket, P's k extra columns (corner 0, after the bv vertex
// dofs) become an orthonormal basis of (tv_j - Ptv_j), j < k, on its owned rows, and every test
// vector's coefficients in that basis go to tvc (whose vertex dofs hold the injection).  Ptv =
// P tvc before the call.  info[w] = 1 where a residual vanishes.  maxrows <= kAugMaxRows.
constexpr int kAugMaxRows = 1024;
void augment(hipStream_t s, const Geom& g, double2* P, const int* rows, const int* nrows, int maxrows,
             const double2* tv, const double2* Ptv, double2* tvc, int nv, int k, int* info);
// P rows scaled by the normalisation (mode 0 TESTVEC, 1 CONST; 2 NONE is a no-op)
void normalise(hipStream_t s, const Geom& g, double2* P, const int* owner, const double2* tv,
               const double2* tvc, int nv, int mode);
void probe_make(hipStream_t s, const Geom& gc, int pt, int px, int ct, int cx, double2* e);
// scatter probe results u [bc][ndof_c] into the coarse stencil [node][25][bc][bc] or dense
void probe_extract(hipStream_t s, const Geom& gc, int pt, int px, int ct, int cx,
                   const double2* u, double2* out, int dense);
void cast_matrix(hipStream_t s, const double2* A, float2* out, int64_t n);
// y += a x (complex arrays, real a)
void axpy_real(hipStream_t s, double2* y, double a, const double2* x, int64_t n);

// ---- Krylov (FP64) -----------------------------------------------------------------------
// Reductions are per-block partials [rhs][nblk][32] (Gram pass: [rhs][nblk][64]); the consumer
// of a reduction adds them in a fixed order itself.  Arnoldi step j with delayed
// reorthogonalisation: gram (slots 0..j with w), lag_control (step j), lag_update; a cycle of m
// steps ends with gram over slots 0..m without w and lag_control for step m.
struct KrylovDims { int64_t n; int nrhs; int nblk; int m; };
constexpr int kMaxKrylovBlocks = 256;          // nblk <= this
// partials of V^H u (u = slot nv-1) and, when w is given, of V^H w, over slots 0..nv-1
void gram(hipStream_t s, const KrylovDims& d, const double2* V, int64_t vsj, int nv, const double2* w,
          double2* part, const RhsState* st);
// finalises Hessenberg column j-1 (rotations, end-of-cycle test) and, with has_w, writes the
// coefficients of lag_update, column j's projections and the direction scale zsc[r][j]
void lag_control(hipStream_t s, const KrylovDims& d, const double2* part, RhsState* st, double2* H,
                 double* cs, double2* sn, double2* g, double2* coef, double* zsc, int j, int has_w,
                 double tol, double inner_tol, int max_iters, double2* hist, int hist_cap);
// slot nv-1 <- final v (when write_v), slot nv <- next direction u, from coef
void lag_update(hipStream_t s, const KrylovDims& d, double2* V, int64_t vsj, int nv, const double2* w,
                const double2* coef, const RhsState* st, int write_v);
// Hessenberg data and convergence settings of one batch (step j set per launch)
struct ArnoldiArgs {
  double2* H;       // [rhs][(m+1) m], H[i][j] at i*m + j
  double* cs;       // [rhs][m]
  double2* sn;      // [rhs][m]
  double2* g;       // [rhs][m+1]
  int j;
  double tol, inner_tol;
  int max_iters;
  double2* hist;
  int hist_cap;
};
// One batch (a lattice's right-hand sides) of the multi-batch Krylov launches, which run the
// step's pass A, control and pass B of several batches in lock step, each batch's work items
// exactly as its own launches would (bitwise the same results).  item0 / rhs0: the batch's
// first block item (prefix of nrhs * nblk) and first rhs item (prefix of nrhs).
struct KrylovSeg {
  KrylovDims dm;
  double2* V;
  int64_t vsj;
  const double2* w;
  double2* part;
  RhsState* st;
  double2* coef;
  double* zsc;
  ArnoldiArgs aa;
  int item0, rhs0;
};
// seg: device array of nseg segments; the same nv, j, has_w and write_v for all of them
void gram_multi(hipStream_t s, const KrylovSeg* seg, int nseg, int total_blocks, int nv);
void lag_control_multi(hipStream_t s, const KrylovSeg* seg, int nseg, int total_rhs, int j, int has_w);
void lag_update_multi(hipStream_t s, const KrylovSeg* seg, int nseg, int total_blocks, int nv, int write_v);
// ||x|| then mode 1: fresh states (x = b); 2: first cycle start (x = r_0); 3: cycle end and
// restart (x = b - D x)
void norm_control(hipStream_t s, const KrylovDims& d, const double2* x, double2* part, RhsState* st,
                  int mode, double2* g, double tol, int max_iters, double2* hist, int hist_cap);
void scale_next(hipStream_t s, const KrylovDims& d, const double2* w, double2* v,
                const RhsState* st);
// st[r] = st2[r] for the slots with admit[r] != 0 (slots joining a running batch)
void merge_states(hipStream_t s, RhsState* st, const RhsState* st2, const int* admit, int cap);
void backsolve_update(hipStream_t s, const KrylovDims& d, RhsState* st, const double2* H,
                      const double2* g, const double* zsc, double2* y, Real zprec, const void* Z,
                      int64_t zstride_j, double2* x);

}  // namespace amamg
