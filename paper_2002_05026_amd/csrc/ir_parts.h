// Bodies of the refinement bookkeeping kernels (Sec. II, dual solution, with
// the FP64 residual of the mixed-precision path): the block-sparse residual
// r = b - K x, column maxima, the eta decision, precision conversions and
// the permutations of the right-hand sides.  Each takes its block
// coordinates explicitly, so that a kernel for one factor and a kernel that
// walks an instance table (one launch for every instance of a batch) share
// them.
#pragma once
#include <hip/hip_runtime.h>

#include "d3m_internal.h"
#include "gemm_engine.h"
#include "launch.h"

namespace d3m {

__device__ __forceinline__ void atomic_max_pos(double* p, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}

// Partial residual products: the workgroup takes row tile t, right-hand
// sides [64 by, 64 by + 64) and chunk bz of the tile's block row, and writes
// P_bz = sum over the chunk's blocks K_IJ X_J (internal rows, RHS fastest;
// zeros for an empty chunk).  Four 16-column FP64 accumulator blocks per
// wave (no register spills at any nrhs), so the registers allow slabs of 16
// columns.  lds: ge_lds_bytes<double, kResKB>().
constexpr int kResCols = 64;
constexpr int kResKB = 16;
__device__ __forceinline__ void residual_tile(const double2* K, const double2* X, double2* P, const UserView& uv,
                                              const RTaskDev t, int nrhs, int by, int bz, lds_char* lds) {
  constexpr int NB = kResCols / 16;
  const int I = t.I;
  const int nI = uv.n[I];
  const int j0 = kResCols * by;
  const int nr = nrhs - j0 < kResCols ? nrhs - j0 : kResCols;
  const int e0 = uv.rsplit[I * (kResSplit + 1) + bz], e1 = uv.rsplit[I * (kResSplit + 1) + bz + 1];
  Acc<double> acc;
  acc.zero();
  for (int e = e0; e < e1; ++e) {
    const RBlkDev b = uv.rblk[e];
    const int nJ = uv.n[b.J];
    Opnd<double> A;
    A.i0 = 0;
    if (b.mode == 0) { A.p = K + b.koff; A.ld = nI; A.mode = OP_SYM; A.i0 = t.r0; }
    else if (b.mode == 1) { A.p = K + b.koff + t.r0; A.ld = nI; A.mode = OP_N; }
    else { A.p = K + b.koff + (int64_t)t.r0 * nJ; A.ld = nJ; A.mode = OP_T; }
    Opnd<double> Bo;
    Bo.p = X + uv.prow0[b.J] * nrhs + j0;
    Bo.ld = nrhs;
    Bo.mode = OP_N;
    Bo.i0 = 0;
    gemm_acc<double, NB, kResKB>(acc, t.sz, nr, nJ, A, nullptr, Bo, lds);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  double2* dst = P + (int64_t)bz * uv.N * nrhs + (uv.prow0[I] + t.r0) * nrhs + j0;
  if (16 * w < t.sz) {
#pragma unroll
    for (int bj = 0; bj < NB; ++bj) {
      const int j = 16 * bj + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + acc_row<double>(lk, v);
        if (i < t.sz && j < nr) {
          double2 r;
          r.x = acc.re[bj][v];
          r.y = acc.im[bj][v];
          dst[(int64_t)i * nrhs + j] = r;
        }
      }
    }
  }
}

// The same partial products with K streamed from global memory straight into
// the MFMA operands (no LDS), for at most 16 NBJ right-hand sides.  With one
// 16-column block of right-hand sides the product does about as many FP64
// flops per byte of K as the matrix cores do per byte of HBM, and the
// LDS-staged form above, one slab of K in flight per workgroup, is then held
// by load latency instead.  Here each wave owns 16 rows of the tile and keeps
// the loads of the next U k-steps (4 columns each) in flight while it
// multiplies the current ones.  The k index of a lane's operands is 4 s + lk
// in both A and B, as in the LDS form; columns beyond the block read a
// clamped address and enter as zeros of A, rows beyond the tile and
// right-hand sides beyond nrhs read clamped addresses and are not stored.
// the direct form is taken for at most kResDirectRhs right-hand sides (one
// block), with kResDirU k-steps of loads in flight
constexpr int kResDirectRhs = 16;
constexpr int kResDirU = 3;
template <int NBJ, int U>
__device__ __forceinline__ void residual_tile_direct(const double2* K, const double2* X, double2* P,
                                                     const UserView& uv, const RTaskDev t, int nrhs, int bz) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int I = t.I;
  const int nI = uv.n[I];
  const int e0 = uv.rsplit[I * (kResSplit + 1) + bz], e1 = uv.rsplit[I * (kResSplit + 1) + bz + 1];
  double2* dst = P + (int64_t)bz * uv.N * nrhs + (uv.prow0[I] + t.r0) * nrhs;
  if (16 * w >= t.sz) return;  // no barrier in this body
  const int ri = 16 * w + lr;
  const int gi = t.r0 + (ri < t.sz ? ri : t.sz - 1);  // this lane's A row inside interface I
  int jc[NBJ];                                        // this lane's B columns
#pragma unroll
  for (int bj = 0; bj < NBJ; ++bj) jc[bj] = 16 * bj + lr < nrhs ? 16 * bj + lr : 0;
  v4d cre[NBJ], cim[NBJ];
#pragma unroll
  for (int bj = 0; bj < NBJ; ++bj) {
    cre[bj] = v4d{0, 0, 0, 0};
    cim[bj] = v4d{0, 0, 0, 0};
  }
  for (int e = e0; e < e1; ++e) {
    const RBlkDev b = uv.rblk[e];
    const int nJ = uv.n[b.J];
    if (nJ <= 0) continue;
    const D3M_GLB cpx<double>* kb = gptr<double>(K + b.koff);
    const D3M_GLB cpx<double>* xb = gptr<double>(X + uv.prow0[b.J] * nrhs);
    const int ng = (nJ + 4 * U - 1) / (4 * U);  // groups of U k-steps
    // one copy of the loop per operand mode: 1 K_IJ (column-major, rows of
    // I contiguous), 2 K_JI^T, 0 the diagonal block from its lower triangle
    auto blk = [&](auto modec) {
      constexpr int MODE = decltype(modec)::value;
      auto aoff = [&](int p) -> int64_t {
        if constexpr (MODE == 1) return gi + (int64_t)p * nI;
        if constexpr (MODE == 2) return (int64_t)gi * nJ + p;
        return gi >= p ? gi + (int64_t)p * nI : p + (int64_t)gi * nI;
      };
      auto fetch = [&](cpx<double>* a, cpx<double>(*x)[NBJ], int g) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int p = 4 * (g * U + u) + lk;
          const int pc = p < nJ ? p : nJ - 1;
          a[u] = kb[aoff(pc)];
#pragma unroll
          for (int bj = 0; bj < NBJ; ++bj) x[u][bj] = xb[(int64_t)pc * nrhs + jc[bj]];
        }
      };
      auto mma = [&](const cpx<double>* a, const cpx<double>(*x)[NBJ], int g) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (4 * (g * U + u) >= nJ) break;  // uniform
          const bool ok = 4 * (g * U + u) + lk < nJ;
          const double ar = ok ? a[u].x : 0.0, ai = ok ? a[u].y : 0.0;
#pragma unroll
          for (int bj = 0; bj < NBJ; ++bj) {
            cre[bj] = mfma16(ar, x[u][bj].x, cre[bj]);
            cre[bj] = mfma16(-ai, x[u][bj].y, cre[bj]);
            cim[bj] = mfma16(ar, x[u][bj].y, cim[bj]);
            cim[bj] = mfma16(ai, x[u][bj].x, cim[bj]);
          }
        }
      };
      cpx<double> a0[U], a1[U];
      cpx<double> x0[U][NBJ], x1[U][NBJ];
      fetch(a0, x0, 0);
      for (int g = 0; g < ng; g += 2) {
        if (g + 1 < ng) fetch(a1, x1, g + 1);
        mma(a0, x0, g);
        if (g + 1 >= ng) break;
        if (g + 2 < ng) fetch(a0, x0, g + 2);
        mma(a1, x1, g + 1);
      }
    };
    if (b.mode == 1) blk(std::integral_constant<int, 1>());
    else if (b.mode == 2) blk(std::integral_constant<int, 2>());
    else blk(std::integral_constant<int, 0>());
  }
#pragma unroll
  for (int bj = 0; bj < NBJ; ++bj) {
    if (16 * bj + lr < nrhs) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + acc_row<double>(lk, v);
        if (i < t.sz) {
          double2 r;
          r.x = cre[bj][v];
          r.y = cim[bj][v];
          dst[(int64_t)i * nrhs + 16 * bj + lr] = r;
        }
      }
    }
  }
}

// R = B - sum_z P_z (internal rows, RHS fastest; B in user layout) and the
// column maxima of |R| into colmax; block bx of gx, 256 threads; cm: 128
// words of LDS.
__device__ __forceinline__ void residual_fin_part(const double2* B, int64_t ld, const double2* P, double2* R,
                                                  double* colmax, const UserView& uv, int nrhs, int bx, int gx,
                                                  unsigned long long* cm) {
  if (threadIdx.x < 128) cm[threadIdx.x] = 0;
  __syncthreads();
  const int64_t tot = uv.N * nrhs;
  for (int64_t e = (int64_t)bx * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gx * blockDim.x) {
    const int64_t q = e / nrhs;
    const int j = (int)(e - q * nrhs);
    double2 r = B[uv.perm[q] + (int64_t)j * ld];
#pragma unroll
    for (int z = 0; z < kResSplit; ++z) {
      const double2 p = P[z * tot + e];
      r.x -= p.x;
      r.y -= p.y;
    }
    R[e] = r;
    double a = sqrt(r.x * r.x + r.y * r.y);
    if (!(a == a)) a = __longlong_as_double(0x7ff0000000000000ll);  // NaN -> inf
    atomicMax(&cm[j], (unsigned long long)__double_as_longlong(a));
  }
  __syncthreads();
  if (threadIdx.x < nrhs && cm[threadIdx.x])
    atomic_max_pos(colmax + threadIdx.x, __longlong_as_double((long long)cm[threadIdx.x]));
}

// Column maxima of |v| for a c128 array: rhs_fastest ? v[row*nrhs + j] :
// v[j*ld + row]; block bx of gx; cm: 128 words of LDS.
__device__ __forceinline__ void colmax_part(const double2* V, int64_t rows, int nrhs, int64_t ld, int rhs_fastest,
                                            double* colmax, int bx, int gx, unsigned long long* cm) {
  if (threadIdx.x < 128) cm[threadIdx.x] = 0;
  __syncthreads();
  const int64_t tot = rows * nrhs;
  for (int64_t e = (int64_t)bx * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gx * blockDim.x) {
    int64_t r;
    int j;
    double2 v;
    if (rhs_fastest) { r = e / nrhs; j = (int)(e - r * nrhs); v = V[e]; }
    else { j = (int)(e / rows); r = e - (int64_t)j * rows; v = V[(int64_t)j * ld + r]; }
    double a = sqrt(v.x * v.x + v.y * v.y);
    if (!(a == a)) a = __longlong_as_double(0x7ff0000000000000ll);
    atomicMax(&cm[j], (unsigned long long)__double_as_longlong(a));
  }
  __syncthreads();
  if (threadIdx.x < nrhs && cm[threadIdx.x])
    atomic_max_pos(colmax + threadIdx.x, __longlong_as_double((long long)cm[threadIdx.x]));
}

// eta_j = rmax_j / (||K|| xmax_j + bmax_j); record max_j eta_j; decide
// (one thread).
__device__ __forceinline__ void ir_check_one(IrCtrl* c, double* rmax, double* xmax, const double* bmax, int nrhs,
                                             int final_step) {
  if (c->stop) return;
  double eta = 0;
  bool nonfinite = false;
  for (int j = 0; j < nrhs; ++j) {
    double den = c->knorm * xmax[j] + bmax[j];
    double e = den > 0 ? rmax[j] / den : rmax[j];
    if (!(e <= 1e300)) nonfinite = true;
    eta = fmax(eta, e);
    rmax[j] = 0;
    xmax[j] = 0;
  }
  const int it = c->it;
  if (it < 32) c->eta_hist[it] = eta;
  c->it = it + 1;
  if (nonfinite) {
    c->status = 2;  // D3M_NONFINITE
    c->stop = 1;
  } else if (eta <= c->tol || final_step == 2) {
    c->stop = 1;
  } else if (final_step || it >= c->max_iter) {
    c->status = 3;  // D3M_IR_NOCONV
    c->stop = 1;
  } else if (it >= 2 && it < 32 && c->eta_hist[it - 2] >= 0 && eta > 0.5 * c->eta_hist[it - 2]) {
    c->status = 3;  // stagnation
    c->stop = 1;
  } else {
    c->iters = it + 1;
  }
}

__device__ __forceinline__ void ir_reset_one(IrCtrl* c, double tol, int max_iter) {
  c->stop = 0;
  c->iters = 0;
  c->status = 0;
  c->it = 0;
  c->tol = tol;
  c->max_iter = max_iter;
  for (int k = 0; k < 32; ++k) c->eta_hist[k] = -1.0;
}

__device__ __forceinline__ void cvt_down_part(const double2* R, float2* W, int64_t n, int bx, int gx) {
  for (int64_t e = (int64_t)bx * blockDim.x + threadIdx.x; e < n; e += (int64_t)gx * blockDim.x) {
    double2 v = R[e];
    W[e] = make_float2((float)v.x, (float)v.y);
  }
}
__device__ __forceinline__ void cvt_up_part(const float2* W, double2* X, int64_t n, int bx, int gx) {
  for (int64_t e = (int64_t)bx * blockDim.x + threadIdx.x; e < n; e += (int64_t)gx * blockDim.x) {
    float2 v = W[e];
    X[e] = make_double2(v.x, v.y);
  }
}
__device__ __forceinline__ void axpy_up_part(const float2* W, double2* X, int64_t n, int bx, int gx) {
  for (int64_t e = (int64_t)bx * blockDim.x + threadIdx.x; e < n; e += (int64_t)gx * blockDim.x) {
    float2 v = W[e];
    double2 x = X[e];
    x.x += v.x;
    x.y += v.y;
    X[e] = x;
  }
}

// W[q*nrhs + j] = B[j*ld + perm[q]] (into the factor's precision) and back.
template <typename T>
__device__ __forceinline__ void perm_in_part(const double2* B, int64_t ld, typename Cplx<T>::type* W,
                                             const int32_t* perm, int64_t N, int nrhs, int bx, int gx) {
  const int64_t tot = N * nrhs;
  for (int64_t e = (int64_t)bx * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gx * blockDim.x) {
    int64_t q = e / nrhs;
    int j = (int)(e - q * nrhs);
    double2 v = B[(int64_t)j * ld + perm[q]];
    typename Cplx<T>::type o;
    o.x = (T)v.x;
    o.y = (T)v.y;
    W[e] = o;
  }
}
__device__ __forceinline__ void perm_out_part(const double2* W, double2* X, int64_t ld, const int32_t* perm,
                                              int64_t N, int nrhs, int bx, int gx) {
  const int64_t tot = N * nrhs;
  for (int64_t e = (int64_t)bx * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gx * blockDim.x) {
    int64_t q = e / nrhs;
    int j = (int)(e - q * nrhs);
    X[(int64_t)j * ld + perm[q]] = W[e];
  }
}

}  // namespace d3m
