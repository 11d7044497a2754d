// Refinement bookkeeping of a batch in one launch per step: the kernels
// walk a table of instances (grid y or z = instance), so an IR step of a
// 32-instance sweep costs a handful of launches instead of a handful per
// instance.  Every instance keeps its own stop flag: a stopped instance's
// workgroups return at once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "d3m_internal.h"
#include "gemm_engine.h"
#include "ir_parts.h"
#include "setup_parts.h"
#include "launch.h"

namespace d3m {

namespace {

__global__ void k_batch_user(BatchIrDev* tab, BatchUserArgs u) {
  const int i = threadIdx.x;
  if (blockIdx.x != 0 || i >= u.count) return;
  BatchIrDev& t = tab[u.base + i];
  t.K = (const double2*)u.K[i];
  t.B = (const double2*)u.B[i];
  t.X = (double2*)u.X[i];
  t.ld = u.ld[i];
}

// grid (workgroups per instance, instances)
__global__ void k_batch_prepare(const BatchIrDev* tab) {
  const BatchIrDev& t = tab[blockIdx.y];
  prepare_part(t.status, t.growth, t.npanel, t.ctrl, t.tol, t.max_iter, blockIdx.x * blockDim.x + threadIdx.x,
               gridDim.x * blockDim.x);
}

// grid (32, all instances' blocks): block y belongs to the last instance
// whose first block (sb0, ascending) is at most y
template <typename T>
__global__ __launch_bounds__(256) void k_batch_scatter(const BatchIrDev* tab, int n) {
  const int y = blockIdx.y;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].sb0 <= y) lo = mid;
    else hi = mid - 1;
  }
  const BatchIrDev& t = tab[lo];
  scatter_part<T>(t.K, (typename Cplx<T>::type*)t.L, t.kp, t.nkp, t.fills, t.part, y - t.sb0, blockIdx.x, gridDim.x);
}

// grid (groups of eight 32-row groups, instances)
__global__ __launch_bounds__(256) void k_batch_knorm(const BatchIrDev* tab) {
  const BatchIrDev& t = tab[blockIdx.y];
  if (8 * (int)blockIdx.x >= t.kn.ngroups) return;
  knorm_part(t.kn, t.ctrl, blockIdx.x);
}

__global__ void k_batch_flags(const BatchIrDev* tab, int n, const int32_t* src) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) *tab[i].flag = *src;
}

// ir reset and zeroed column maxima (one block per instance)
__global__ void k_batch_start(BatchIrDev* tab) {
  const BatchIrDev& t = tab[blockIdx.x];
  if (threadIdx.x == 0) ir_reset_one(t.ctrl, t.tol, t.max_iter);
  for (int i = threadIdx.x; i < 3 * 128; i += blockDim.x) t.rmax[i] = 0;
}

// column maxima of B (user layout) into bmax
__global__ void k_batch_colmax_b(const BatchIrDev* tab) {
  const BatchIrDev& t = tab[blockIdx.y];
  __shared__ unsigned long long cm[128];
  colmax_part(t.B, t.uv.N, t.nrhs, t.ld, 0, t.bmax, blockIdx.x, gridDim.x, cm);
}

template <typename T>
__global__ void k_batch_perm_in(const BatchIrDev* tab) {
  const BatchIrDev& t = tab[blockIdx.y];
  perm_in_part<T>(t.B, t.ld, (typename Cplx<T>::type*)t.W, t.uv.perm, t.uv.N, t.nrhs, blockIdx.x, gridDim.x);
}

__global__ void k_batch_cvt_up(const BatchIrDev* tab) {
  const BatchIrDev& t = tab[blockIdx.y];
  cvt_up_part((const float2*)t.W, t.X64, t.uv.N * t.nrhs, blockIdx.x, gridDim.x);
}

// grid (row tiles, RHS chunks x kResSplit, instances)
__global__ __launch_bounds__(kThreads) void k_batch_residual(const BatchIrDev* tab, int ny, int prec) {
  __shared__ __attribute__((aligned(16))) char lds[ge_lds_bytes<double, kResKB>()];
  const BatchIrDev& t = tab[blockIdx.z];
  if (t.ctrl->stop || t.nrhs <= kResDirectRhs) return;  // those take k_batch_residual_direct
  const int by = blockIdx.y % ny, bz = blockIdx.y / ny;
  if ((int)blockIdx.x >= t.nrt || kResCols * by >= t.nrhs) return;
  const double2* X = prec == 0 ? (const double2*)t.W : t.X64;
  residual_tile(t.K, X, t.P64, t.uv, t.rt[blockIdx.x], t.nrhs, by, bz, (lds_char*)lds);
}

// grid (row tiles, kResSplit, instances); instances of at most kResDirectRhs
// right-hand sides, as in the single-factor residual
__global__ __launch_bounds__(kThreads) void k_batch_residual_direct(const BatchIrDev* tab, int prec) {
  const BatchIrDev& t = tab[blockIdx.z];
  if (t.ctrl->stop || t.nrhs > kResDirectRhs || (int)blockIdx.x >= t.nrt) return;
  const double2* X = prec == 0 ? (const double2*)t.W : t.X64;
  const UserView uv = t.uv;
  const RTaskDev rt = t.rt[blockIdx.x];
  residual_tile_direct<1, kResDirU>(t.K, X, t.P64, uv, rt, t.nrhs, blockIdx.y);
}

__global__ void k_batch_residual_fin(const BatchIrDev* tab) {
  const BatchIrDev& t = tab[blockIdx.y];
  if (t.ctrl->stop) return;
  __shared__ unsigned long long cm[128];
  residual_fin_part(t.B, t.ld, t.P64, t.R64, t.rmax, t.uv, t.nrhs, blockIdx.x, gridDim.x, cm);
}

__global__ void k_batch_colmax_x(const BatchIrDev* tab, int prec) {
  const BatchIrDev& t = tab[blockIdx.y];
  if (t.ctrl->stop) return;
  __shared__ unsigned long long cm[128];
  const double2* X = prec == 0 ? (const double2*)t.W : t.X64;
  colmax_part(X, t.uv.N, t.nrhs, 0, 1, t.xmax, blockIdx.x, gridDim.x, cm);
}

__global__ void k_batch_ir_check(BatchIrDev* tab, int final_step) {
  const BatchIrDev& t = tab[blockIdx.x];
  if (threadIdx.x == 0) ir_check_one(t.ctrl, t.rmax, t.xmax, t.bmax, t.nrhs, final_step);
}

__global__ void k_batch_cvt_down(const BatchIrDev* tab) {
  const BatchIrDev& t = tab[blockIdx.y];
  if (t.ctrl->stop) return;
  cvt_down_part(t.R64, (float2*)t.W, t.uv.N * t.nrhs, blockIdx.x, gridDim.x);
}

__global__ void k_batch_axpy_up(const BatchIrDev* tab) {
  const BatchIrDev& t = tab[blockIdx.y];
  if (t.ctrl->stop) return;
  axpy_up_part((const float2*)t.W, t.X64, t.uv.N * t.nrhs, blockIdx.x, gridDim.x);
}

__global__ void k_batch_perm_out(const BatchIrDev* tab, int prec) {
  const BatchIrDev& t = tab[blockIdx.y];
  const double2* W = prec == 0 ? (const double2*)t.W : t.X64;
  perm_out_part(W, t.X, t.ld, t.uv.perm, t.uv.N, t.nrhs, blockIdx.x, gridDim.x);
}

int blocks_for(int64_t maxtot, int cap) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((maxtot + 255) / 256, cap));
}

}  // namespace

hipError_t launch_batch_user(BatchIrDev* tab, int n, const void* const* K, const void* const* B, void* const* X,
                             const int64_t* ld, hipStream_t s) {
  for (int base = 0; base < n; base += kBatchUserMax) {
    BatchUserArgs u;
    u.base = base;
    u.count = std::min(kBatchUserMax, n - base);
    for (int i = 0; i < u.count; ++i) {
      u.K[i] = K[base + i];
      u.B[i] = B[base + i];
      u.X[i] = X[base + i];
      u.ld[i] = ld[base + i];
    }
    hipLaunchKernelGGL(k_batch_user, dim3(1), dim3(64), 0, s, tab, u);
  }
  return hipGetLastError();
}

hipError_t launch_batch_setup(BatchIrDev* tab, int n, int prec, int totnb, int maxkng, int maxpanel, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_prepare, dim3(std::max(1, (maxpanel + 255) / 256), n), dim3(256), 0, s, tab);
  if (totnb > 0) {
    if (prec == 0) hipLaunchKernelGGL(k_batch_scatter<double>, dim3(32, totnb), dim3(256), 0, s, tab, n);
    else hipLaunchKernelGGL(k_batch_scatter<float>, dim3(32, totnb), dim3(256), 0, s, tab, n);
  }
  if (maxkng > 0) hipLaunchKernelGGL(k_batch_knorm, dim3((maxkng + 7) / 8, n), dim3(256), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_batch_flags(BatchIrDev* tab, int n, const int32_t* src, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_flags, dim3((n + 63) / 64), dim3(64), 0, s, tab, n, src);
  return hipGetLastError();
}

hipError_t launch_batch_begin(BatchIrDev* tab, int n, int prec, int64_t maxtot, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_start, dim3(n), dim3(128), 0, s, tab);
  hipLaunchKernelGGL(k_batch_colmax_b, dim3(blocks_for(maxtot, 2048), n), dim3(256), 0, s, tab);
  if (prec == 0)
    hipLaunchKernelGGL(k_batch_perm_in<double>, dim3(blocks_for(maxtot, 4096), n), dim3(256), 0, s, tab);
  else
    hipLaunchKernelGGL(k_batch_perm_in<float>, dim3(blocks_for(maxtot, 4096), n), dim3(256), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_batch_cvt_up(BatchIrDev* tab, int n, int64_t maxtot, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_cvt_up, dim3(blocks_for(maxtot, 8192), n), dim3(256), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_batch_check(BatchIrDev* tab, int n, int prec, int maxnrt, int minnrhs, int maxnrhs,
                              int64_t maxtot, int final_step, hipStream_t s) {
  if (maxnrhs > 128) return hipErrorInvalidValue;
  const int ny = (maxnrhs + kResCols - 1) / kResCols;
  if (minnrhs <= kResDirectRhs)
    hipLaunchKernelGGL(k_batch_residual_direct, dim3(maxnrt, kResSplit, n), dim3(kThreads), 0, s, tab, prec);
  if (maxnrhs > kResDirectRhs)
    hipLaunchKernelGGL(k_batch_residual, dim3(maxnrt, ny * kResSplit, n), dim3(kThreads), 0, s, tab, ny, prec);
  hipLaunchKernelGGL(k_batch_residual_fin, dim3(blocks_for(maxtot, 4096), n), dim3(256), 0, s, tab);
  hipLaunchKernelGGL(k_batch_colmax_x, dim3(blocks_for(maxtot, 2048), n), dim3(256), 0, s, tab, prec);
  hipLaunchKernelGGL(k_batch_ir_check, dim3(n), dim3(64), 0, s, tab, final_step);
  return hipGetLastError();
}

hipError_t launch_batch_cvt_down(BatchIrDev* tab, int n, int64_t maxtot, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_cvt_down, dim3(blocks_for(maxtot, 8192), n), dim3(256), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_batch_axpy_up(BatchIrDev* tab, int n, int64_t maxtot, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_axpy_up, dim3(blocks_for(maxtot, 8192), n), dim3(256), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_batch_perm_out(BatchIrDev* tab, int n, int prec, int64_t maxtot, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_perm_out, dim3(blocks_for(maxtot, 4096), n), dim3(256), 0, s, tab, prec);
  return hipGetLastError();
}

}  // namespace d3m
