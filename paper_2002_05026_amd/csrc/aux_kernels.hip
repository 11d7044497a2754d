// Stream-ordered kernels around the DAG launches: scatter/convert of K into
// panel storage, permutation of right-hand sides into elimination order,
// the FP64 block-sparse residual r = b - K x with column norms, the norm of
// K, refinement bookkeeping, precision conversion, and the gradient blocks
// dK = -sym(Lambda X^T) on K's pattern.
#include <hip/hip_runtime.h>

#include "d3m_internal.h"
#include "gemm_engine.h"
#include "launch.h"
#include "ir_parts.h"
#include "setup_parts.h"

namespace d3m {

// ---------------------------------------------------------------- prepare
__global__ void k_prepare(int32_t* status, float* growth, int npanel, IrCtrl* ctrl, double tol, int max_iter) {
  prepare_part(status, growth, npanel, ctrl, tol, max_iter, blockIdx.x * blockDim.x + threadIdx.x,
               gridDim.x * blockDim.x);
}

hipError_t launch_prepare(int32_t* status, float* growth, int npanel, IrCtrl* ctrl, double tol, int max_iter,
                          hipStream_t s) {
  int blocks = (npanel + 255) / 256;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_prepare, dim3(blocks), dim3(256), 0, s, status, growth, npanel, ctrl, tol, max_iter);
  return hipGetLastError();
}

// ---------------------------------------------------------------- scatter
template <typename T>
__global__ __launch_bounds__(256) void k_scatter(const double2* K, typename Cplx<T>::type* L, const KPlaceDev* kp,
                                                 int nkp, const KPlaceDev* fills, double* part) {
  scatter_part<T>(K, L, kp, nkp, fills, part, blockIdx.y, blockIdx.x, gridDim.x);
}

hipError_t launch_scatter(const void* K, void* L, const KPlaceDev* kp, int nkp, const KPlaceDev* fills,
                          int nfill, double* part, int prec, hipStream_t s) {
  int nb = nkp + nfill;
  if (nb == 0) return hipSuccess;
  dim3 grid(32, nb);
  if (prec == 0)
    hipLaunchKernelGGL(k_scatter<double>, grid, dim3(256), 0, s, (const double2*)K, (double2*)L, kp, nkp, fills, part);
  else
    hipLaunchKernelGGL(k_scatter<float>, grid, dim3(256), 0, s, (const double2*)K, (float2*)L, kp, nkp, fills, part);
  return hipGetLastError();
}

// ---------------------------------------------------------------- permutation
template <typename T>
__global__ void k_perm_in(const double2* B, int64_t ld, typename Cplx<T>::type* W, const int32_t* perm,
                          int64_t N, int nrhs, const int32_t* skip) {
  if (skip && *skip) return;
  perm_in_part<T>(B, ld, W, perm, N, nrhs, blockIdx.x, gridDim.x);
}

hipError_t launch_perm_in(const void* B, int64_t ld, void* W, int prec, const UserView& uv, int nrhs,
                          const int32_t* skip, hipStream_t s) {
  int64_t tot = uv.N * nrhs;
  int blocks = (int)std::min<int64_t>((tot + 255) / 256, 4096);
  if (prec == 0)
    hipLaunchKernelGGL(k_perm_in<double>, dim3(blocks), dim3(256), 0, s, (const double2*)B, ld, (double2*)W, uv.perm, uv.N, nrhs, skip);
  else
    hipLaunchKernelGGL(k_perm_in<float>, dim3(blocks), dim3(256), 0, s, (const double2*)B, ld, (float2*)W, uv.perm, uv.N, nrhs, skip);
  return hipGetLastError();
}

__global__ void k_perm_out(const double2* W, double2* X, int64_t ld, const int32_t* perm, int64_t N, int nrhs) {
  perm_out_part(W, X, ld, perm, N, nrhs, blockIdx.x, gridDim.x);
}

hipError_t launch_perm_out(const void* W, void* X, int64_t ld, const UserView& uv, int nrhs, hipStream_t s) {
  int64_t tot = uv.N * nrhs;
  int blocks = (int)std::min<int64_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_perm_out, dim3(blocks), dim3(256), 0, s, (const double2*)W, (double2*)X, ld, uv.perm, uv.N, nrhs);
  return hipGetLastError();
}

// Rows [q0, q1) (internal order) only: W[q*nrhs + j] = B[j*ld + perm[q]]
// (in) or X[j*ld + perm[q]] = W[q*nrhs + j] (out), complex128.
__global__ void k_perm_rows(const double2* src, int64_t lds, double2* dst, int64_t ldd, const int32_t* perm,
                            int64_t q0, int64_t q1, int nrhs, int out) {
  const int64_t tot = (q1 - q0) * nrhs;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = q0 + e / nrhs;
    const int j = (int)(e % nrhs);
    if (out) dst[(int64_t)j * ldd + perm[q]] = src[q * nrhs + j];
    else dst[q * nrhs + j] = src[(int64_t)j * lds + perm[q]];
  }
}

hipError_t launch_perm_rows(const void* src, int64_t lds, void* dst, int64_t ldd, const UserView& uv, int64_t q0,
                            int64_t q1, int nrhs, int out, hipStream_t s) {
  const int64_t tot = (q1 - q0) * nrhs;
  if (tot <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_perm_rows, dim3(blocks), dim3(256), 0, s, (const double2*)src, lds, (double2*)dst, ldd,
                     uv.perm, q0, q1, nrhs, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- reduced matrix out
// Blocks of the reduced matrix from panel storage (complex128), one block
// per blockIdx.y: K(i, j) = panel(i, j) (trans 0) or panel(j, i) (trans 1);
// a diagonal block (rows == cols, trans 0, the first nred entries) is read
// from its lower triangle and written whole, symmetric.
__global__ __launch_bounds__(256) void k_gather_red(const double2* L, double2* K, const KPlaceDev* kg, int ndiag) {
  const int b = blockIdx.y;
  const KPlaceDev P = kg[b];
  const int Kr = P.trans ? P.cols : P.rows, Kc = P.trans ? P.rows : P.cols;  // K block is Kr x Kc
  const int64_t tot = (int64_t)Kr * Kc;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % Kr), j = (int)(e / Kr);
    int r = P.trans ? j : i, c = P.trans ? i : j;  // panel (r, c)
    if (b < ndiag && r < c) { const int t = r; r = c; c = t; }
    K[P.dst + e] = L[P.src + r + (int64_t)c * P.ld_dst];
  }
}

hipError_t launch_gather_red(const void* L, void* K, const KPlaceDev* kg, int nkg, int ndiag, int maxelems,
                             hipStream_t s) {
  if (nkg == 0) return hipSuccess;
  const int bx = std::max(1, std::min(64, (maxelems + 255) / 256));
  hipLaunchKernelGGL(k_gather_red, dim3(bx, nkg), dim3(256), 0, s, (const double2*)L, (double2*)K, kg, ndiag);
  return hipGetLastError();
}

// ---------------------------------------------------------------- port projections
// S[p + q*nports] = sum_i M[i + p*ldm] U[i + q*ldu] (bilinear), one
// workgroup per (p, q); fixed-order partial sums, then a fixed tree.
__global__ __launch_bounds__(256) void k_ports(const double2* M, int64_t ldm, const double2* U, int64_t ldu,
                                               int64_t N, int nports, double2* S) {
  __shared__ double2 red[256];
  const int p = blockIdx.x, q = blockIdx.y;
  double2 acc = {0, 0};
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
    const double2 m = M[i + p * ldm], u = U[i + q * ldu];
    acc.x += m.x * u.x - m.y * u.y;
    acc.y += m.x * u.y + m.y * u.x;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[threadIdx.x].x += red[threadIdx.x + w].x;
      red[threadIdx.x].y += red[threadIdx.x + w].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) S[p + (int64_t)q * nports] = red[0];
}

hipError_t launch_ports(const void* M, int64_t ldm, const void* U, int64_t ldu, int64_t N, int nports, int nrhs,
                        void* S, hipStream_t s) {
  if (nports <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ports, dim3(nports, nrhs), dim3(256), 0, s, (const double2*)M, ldm, (const double2*)U, ldu, N,
                     nports, (double2*)S);
  return hipGetLastError();
}

// ---------------------------------------------------------------- residual
// (the bodies are in ir_parts.h, shared with the batched launches)
__global__ __launch_bounds__(kThreads) void k_residual(const double2* K, const double2* X, double2* P, UserView uv,
                                                  const RTaskDev* rt, int nrhs, const int32_t* skip) {
  __shared__ __attribute__((aligned(16))) char lds[ge_lds_bytes<double, kResKB>()];
  if (skip && *skip) return;
  residual_tile(K, X, P, uv, rt[blockIdx.x], nrhs, blockIdx.y, blockIdx.z, (lds_char*)lds);
}

// The same with K read straight into the matrix-core operands (no LDS):
// NBJ 16-column blocks of right-hand sides, U k-steps of loads in flight
template <int NBJ, int U>
__global__ __launch_bounds__(kThreads) void k_residual_direct(const double2* K, const double2* X, double2* P,
                                                         UserView uv, const RTaskDev* rt, int nrhs,
                                                         const int32_t* skip) {
  if (skip && *skip) return;
  residual_tile_direct<NBJ, U>(K, X, P, uv, rt[blockIdx.x], nrhs, blockIdx.z);
}

// R = B - sum_z P_z (internal rows, RHS fastest; B in user layout) and the
// column maxima of |R| into colmax.
__global__ void k_residual_fin(const double2* B, int64_t ld, const double2* P, double2* R, double* colmax,
                               UserView uv, int nrhs, const int32_t* skip) {
  if (skip && *skip) return;
  __shared__ unsigned long long cm[128];
  residual_fin_part(B, ld, P, R, colmax, uv, nrhs, blockIdx.x, gridDim.x, cm);
}

hipError_t launch_residual(const void* K, const void* B, int64_t ld, const void* X64, void* R64, void* P,
                           double* colmax, const UserView& uv, const RTaskDev* rt, int nrt, int nrhs,
                           const int32_t* skip, hipStream_t s) {
  if (nrhs > 128) return hipErrorInvalidValue;
  const int ny = (nrhs + kResCols - 1) / kResCols;
  // (four blocks of right-hand sides in the direct form measured within 3%
  // of the LDS form, where the matrix cores rather than latency bound it)
  if (nrhs <= kResDirectRhs)
    hipLaunchKernelGGL((k_residual_direct<1, kResDirU>), dim3(nrt, 1, kResSplit), dim3(kThreads), 0, s,
                       (const double2*)K, (const double2*)X64, (double2*)P, uv, rt, nrhs, skip);
  else
    hipLaunchKernelGGL(k_residual, dim3(nrt, ny, kResSplit), dim3(kThreads), 0, s, (const double2*)K,
                       (const double2*)X64, (double2*)P, uv, rt, nrhs, skip);
  const int64_t tot = uv.N * nrhs;
  const int blocks = (int)std::min<int64_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_residual_fin, dim3(blocks), dim3(256), 0, s, (const double2*)B, ld, (const double2*)P,
                     (double2*)R64, colmax, uv, nrhs, skip);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_knorm(KnormDev kn, IrCtrl* ctrl) { knorm_part(kn, ctrl, blockIdx.x); }

hipError_t launch_knorm(const KnormDev& kn, IrCtrl* ctrl, hipStream_t s) {
  if (kn.ngroups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_knorm, dim3((kn.ngroups + 7) / 8), dim3(256), 0, s, kn, ctrl);
  return hipGetLastError();
}

// Column maxima of |v| for a c128 array: rhs_fastest ? v[row*nrhs + j] : v[j*ld + row].
__global__ void k_colmax(const double2* V, int64_t rows, int nrhs, int64_t ld, int rhs_fastest, double* colmax,
                         const int32_t* skip) {
  if (skip && *skip) return;
  __shared__ unsigned long long cm[128];
  colmax_part(V, rows, nrhs, ld, rhs_fastest, colmax, blockIdx.x, gridDim.x, cm);
}

hipError_t launch_colmax(const void* V, int64_t rows, int nrhs, int64_t ld, int rhs_fastest, double* colmax,
                         const int32_t* skip, hipStream_t s) {
  int64_t tot = rows * nrhs;
  int blocks = (int)std::min<int64_t>((tot + 255) / 256, 2048);
  hipLaunchKernelGGL(k_colmax, dim3(blocks), dim3(256), 0, s, (const double2*)V, rows, nrhs, ld, rhs_fastest, colmax, skip);
  return hipGetLastError();
}

__global__ void k_ir_check(IrCtrl* c, double* rmax, double* xmax, const double* bmax, int nrhs, int final_step) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  ir_check_one(c, rmax, xmax, bmax, nrhs, final_step);
}

__global__ void k_ir_reset(IrCtrl* c, double tol, int max_iter) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  ir_reset_one(c, tol, max_iter);
}

hipError_t launch_ir_reset(IrCtrl* ctrl, double tol, int max_iter, hipStream_t s) {
  hipLaunchKernelGGL(k_ir_reset, dim3(1), dim3(64), 0, s, ctrl, tol, max_iter);
  return hipGetLastError();
}

hipError_t launch_ir_check(IrCtrl* ctrl, double* rmax, double* xmax, const double* bmax, int nrhs,
                           int final_step, hipStream_t s) {
  hipLaunchKernelGGL(k_ir_check, dim3(1), dim3(64), 0, s, ctrl, rmax, xmax, bmax, nrhs, final_step);
  return hipGetLastError();
}

__global__ void k_cvt_down(const double2* R, float2* W, int64_t n, const int32_t* skip) {
  if (skip && *skip) return;
  cvt_down_part(R, W, n, blockIdx.x, gridDim.x);
}
__global__ void k_cvt_up(const float2* W, double2* X, int64_t n) { cvt_up_part(W, X, n, blockIdx.x, gridDim.x); }
__global__ void k_axpy_up(const float2* W, double2* X, int64_t n, const int32_t* skip) {
  if (skip && *skip) return;
  axpy_up_part(W, X, n, blockIdx.x, gridDim.x);
}
static int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }
hipError_t launch_cvt_down(const void* R64, void* W32, int64_t n, const int32_t* skip, hipStream_t s) {
  hipLaunchKernelGGL(k_cvt_down, dim3(grid_for(n)), dim3(256), 0, s, (const double2*)R64, (float2*)W32, n, skip);
  return hipGetLastError();
}
hipError_t launch_cvt_up(const void* W32, void* X64, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_cvt_up, dim3(grid_for(n)), dim3(256), 0, s, (const float2*)W32, (double2*)X64, n);
  return hipGetLastError();
}
hipError_t launch_axpy_up(const void* W32, void* X64, int64_t n, const int32_t* skip, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_up, dim3(grid_for(n)), dim3(256), 0, s, (const float2*)W32, (double2*)X64, n, skip);
  return hipGetLastError();
}
__global__ void k_zero_f64(double* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}
hipError_t launch_zero_f64(double* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- dK
// dK(I,J) tile = -1/2 sum_k (lam_I x_J^T + x_I lam_J^T); user layout vectors.
// stored: the gradient with respect to the stored entries of the K buffer
// instead, i.e. each value times the number of entries of the symmetric K
// it stands for: 2 for an off-diagonal block (K_IJ and its mirror K_JI), and
// inside a diagonal block (read from its lower triangle) 2 below the
// diagonal, 1 on it, 0 above.
__global__ __launch_bounds__(kThreads) void k_dk(const double2* Lam, const double2* X, int64_t ld, int nrhs, double2* dK,
                                            UserView uv, const DkTaskDev* dt, int stored) {
  __shared__ __attribute__((aligned(16))) char lds[ge_lds_bytes_dma<double>()];
  const DkTaskDev t = dt[blockIdx.x];
  const int64_t ri = uv.row0[t.I] + t.r0, rj = uv.row0[t.J] + t.c0;
  Acc<double, true> acc;
  acc.zero();
  Opnd<double> A, B;
  A.mode = B.mode = OP_N;
  A.i0 = B.i0 = 0;
  A.ld = B.ld = ld;
  A.p = Lam + ri;
  B.p = X + rj;
  gemm_acc<double, 8, GeKB<double>::KB, OP_N, true>(acc, t.m, t.n, nrhs, A, nullptr, B, (lds_char*)lds);
  A.p = X + ri;
  B.p = Lam + rj;
  gemm_acc<double, 8, GeKB<double>::KB, OP_N, true>(acc, t.m, t.n, nrhs, A, nullptr, B, (lds_char*)lds);
  if (stored) {
    // item (bj, v) of lane (lr, lk) in wave w is element (16w + lr, 16bj + acc_row(lk, v)) of the tile
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lk = lane >> 4;
    const int gi = t.r0 + 16 * w + lr;
#pragma unroll
    for (int bj = 0; bj < 8; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gj = t.c0 + 16 * bj + acc_row<double>(lk, v);
        const double wgt = t.I != t.J ? 2.0 : (gi > gj ? 2.0 : (gi == gj ? 1.0 : 0.0));
        acc.re[bj][v] *= wgt;
        acc.im[bj][v] *= wgt;
      }
  }
  Out<double> o;
  const int nI = uv.n[t.I];
  o.dst = dK + t.koff + t.r0 + (int64_t)t.c0 * nI;
  o.rs = 1;
  o.cs = nI;
  o.src = nullptr;
  o.srs = o.scs = 0;
  o.alpha = -0.5;
  o.beta = 0;
  o.rowdiv = o.coldiv = nullptr;
  o.dst2 = nullptr;
  gemm_store<double>(acc, t.m, t.n, o);
}

hipError_t launch_dk(const void* Lam, const void* X, int64_t ld, int nrhs, void* dK, const UserView& uv,
                     const DkTaskDev* dt, int ndt, int stored, hipStream_t s) {
  if (ndt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dk, dim3(ndt), dim3(kThreads), 0, s, (const double2*)Lam, (const double2*)X, ld, nrhs,
                     (double2*)dK, uv, dt, stored);
  return hipGetLastError();
}

// out = 1 when every instance's refinement has stopped.
__global__ void k_all_stop(IrCtrl* const* ctrls, int n, int32_t* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int all = 1;
  for (int i = 0; i < n; ++i) all &= ctrls[i]->stop ? 1 : 0;
  *out = all;
}

hipError_t launch_all_stop(IrCtrl* const* ctrls, int n, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_all_stop, dim3(1), dim3(64), 0, s, ctrls, n, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- engine check
template <typename T>
__global__ __launch_bounds__(kThreads) void k_debug_gemm(int m, int n, int k, int amode, int i0,
                                                         const typename Cplx<T>::type* A, int64_t lda,
                                                         const typename Cplx<T>::type* d,
                                                         const typename Cplx<T>::type* B, int64_t ldb,
                                                         typename Cplx<T>::type* C, int64_t ldc, T alpha, T beta) {
  __shared__ __attribute__((aligned(16))) char lds[ge_lds_bytes<T>()];
  Acc<T> acc;
  acc.zero();
  Opnd<T> a, b;
  a.p = A;
  a.ld = lda;
  a.mode = amode;
  a.i0 = i0;
  b.p = B;
  b.ld = ldb;
  b.mode = OP_N;
  b.i0 = 0;
  gemm_acc<T>(acc, m, n, k, a, d, b, (lds_char*)lds);
  Out<T> o;
  o.dst = C;
  o.rs = 1;
  o.cs = ldc;
  o.src = beta != (T)0 ? C : nullptr;
  o.srs = 1;
  o.scs = ldc;
  o.alpha = alpha;
  o.beta = beta;
  o.rowdiv = o.coldiv = nullptr;
  o.dst2 = nullptr;
  gemm_store<T>(acc, m, n, o);
}

hipError_t launch_debug_gemm(int prec, int m, int n, int k, int amode, int i0, const void* A, int64_t lda,
                             const void* d, const void* B, int64_t ldb, void* C, int64_t ldc, double alpha,
                             double beta, hipStream_t s) {
  if (prec == 0)
    hipLaunchKernelGGL(k_debug_gemm<double>, dim3(1), dim3(kThreads), 0, s, m, n, k, amode, i0, (const double2*)A,
                       lda, (const double2*)d, (const double2*)B, ldb, (double2*)C, ldc, alpha, beta);
  else
    hipLaunchKernelGGL(k_debug_gemm<float>, dim3(1), dim3(kThreads), 0, s, m, n, k, amode, i0, (const float2*)A,
                       lda, (const float2*)d, (const float2*)B, ldb, (float2*)C, ldc, (float)alpha, (float)beta);
  return hipGetLastError();
}

// ---------------------------------------------------------------- GEMM timing
// Candidate engine paths, timed on repeated products with one private
// region of 3 * 128 * 512 elements per workgroup:
//   0: an update tile, 128 x 128 x 512 (A, B private), the path the factor's
//      updates take (direct loads for complex64, register slabs for
//      complex128);
//   1: the same product through register slabs of half the depth (complex64:
//      register slabs instead of direct loads);
//   2: a solve tile, 64 x 64 x 448 (B shared by all workgroups, as the
//      right-hand-side block of a source panel; A one of five private tiles
//      in turn, together larger than the last-level cache, so that A
//      streams from HBM as the factor does in a solve), whole k per wave;
//   3: the solve tile with k split over the two halves of the workgroup.

template <typename T, int V>
__global__ __launch_bounds__(kThreads) void k_gemm_bench(typename Cplx<T>::type* buf, int reps) {
  typedef typename Cplx<T>::type C;
  __shared__ __attribute__((aligned(16))) char lds[ge_lds_bytes_dma<T>()];
  static_assert(ge_lds_bytes<T, GeKB<T>::KB>() <= ge_lds_bytes_dma<T>(), "register path LDS");
  C* base = buf + (int64_t)blockIdx.x * (3 * 128 * 512);
  Acc<T> acc;
  for (int r = 0; r < reps; ++r) {
    acc.zero();
    Opnd<T> A, B;
    Out<T> o;
    o.rowdiv = o.coldiv = nullptr;
    o.dst2 = nullptr;
    o.alpha = -1;
    o.beta = 1;
    A.mode = OP_N;
    A.i0 = 0;
    if constexpr (V <= 1) {
      A.p = base;
      A.ld = 128;
      B = A;
      B.p = base + 128 * 512;
      if constexpr (V == 0) gemm_acc<T, 8, GeKB<T>::KB, OP_N, true>(acc, 128, 128, 512, A, nullptr, B, (lds_char*)lds);
      else gemm_acc<T, 8, GeKB<T>::KB / 2, OP_N, false>(acc, 128, 128, 512, A, nullptr, B, (lds_char*)lds);
      o.dst = base + 2 * 128 * 512;
      o.rs = 1;
      o.cs = 128;
      o.src = o.dst;
      o.srs = 1;
      o.scs = 128;
      gemm_store<T>(acc, 128, 128, o);
    } else {
      // region: A tiles [0, 5 * 64 * 448), C, then (workgroup 0's) B
      constexpr int kA = 64 * 448;
      A.p = base + (r % 5) * kA;
      A.ld = 64;
      B = A;
      B.p = buf + 5 * kA + 64 * 64;
      gemm_acc<T, 8, GeKB<T>::KB, OP_N, true, false, false, true, V == 3>(acc, 64, 64, 448, A, nullptr, B,
                                                                         (lds_char*)lds);
      o.dst = base + 5 * kA;
      o.rs = 64;
      o.cs = 1;
      o.src = o.dst;
      o.srs = 64;
      o.scs = 1;
      gemm_store<T>(acc, 64, 64, o);
    }
  }
}

hipError_t launch_gemm_bench(int prec, void* buf, int reps, int variant, hipStream_t s) {
  auto go = [&](auto tt, auto vv) {
    typedef decltype(tt) T;
    constexpr int V = decltype(vv)::value;
    hipLaunchKernelGGL((k_gemm_bench<T, V>), dim3(256), dim3(kThreads), 0, s, (typename Cplx<T>::type*)buf, reps);
  };
  auto pick = [&](auto tt) {
    switch (variant) {
      case 0: go(tt, std::integral_constant<int, 0>()); break;
      case 1: go(tt, std::integral_constant<int, 1>()); break;
      case 2: go(tt, std::integral_constant<int, 2>()); break;
      default: go(tt, std::integral_constant<int, 3>()); break;
    }
  };
  if (prec == 0) pick(double());
  else pick(float());
  return hipGetLastError();
}

}  // namespace d3m
