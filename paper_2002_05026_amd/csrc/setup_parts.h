// Set-up steps of a factorization (state reset, scatter/convert of K into
// the factor storage, ||K||_inf), as device functions over a workgroup's
// share of the work, so that one instance's kernels and a batch's kernels
// (instance = a grid dimension) run the same code.
#pragma once
#include <hip/hip_runtime.h>

#include "d3m_internal.h"
#include "ir_parts.h"

namespace d3m {

// Failure state, growth records and refinement control of one factor:
// thread i of stride (i = 0 also resets the single fields).
__device__ __forceinline__ void prepare_part(int32_t* status, float* growth, int npanel, IrCtrl* ctrl, double tol,
                                             int max_iter, int i, int stride) {
  if (i == 0) {
    status[0] = 0x7fffffff;
    status[1] = 0;
    status[2] = 0;
    if (ctrl) {
      ctrl->stop = 0;
      ctrl->iters = 0;
      ctrl->status = 0;
      ctrl->it = 0;
      ctrl->knorm = 0;
      ctrl->tol = tol;
      ctrl->max_iter = max_iter;
      for (int k = 0; k < 32; ++k) ctrl->eta_hist[k] = -1.0;
    }
  }
  for (; i < npanel; i += stride) {
    growth[2 * i] = __int_as_float(0x7f800000);
    growth[2 * i + 1] = 0.f;
  }
}

// Scatter/convert of one block of K into the factor storage: b indexes the
// K placements first, then the fill blocks (zeroed); 32x32 tiles of a K
// block (the elements of a fill block) are spread over the bx-th of gx
// workgroups (256 threads).  Transposed blocks go through LDS.
template <typename T>
__device__ __forceinline__ void scatter_part(const double2* K, typename Cplx<T>::type* L, const KPlaceDev* kp,
                                             int nkp, const KPlaceDev* fills, int b, int bx, int gx) {
  typedef typename Cplx<T>::type C;
  __shared__ double2 tileb[32][33];
  const bool fill = b >= nkp;
  const KPlaceDev P = fill ? fills[b - nkp] : kp[b];
  if (fill) {
    // zeros, 16 bytes per store (a row pair in complex64): a fill block
    // starts at an even row of an even-height panel, and the row after an
    // odd last row is the panel's unused padding row
    constexpr int PER = 16 / (int)sizeof(C);
    const int64_t rp = (P.rows + PER - 1) / PER, tot = rp * P.cols;
    const float4 z = {0.f, 0.f, 0.f, 0.f};
    for (int64_t e = (int64_t)bx * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gx * blockDim.x) {
      const int64_t c = e / rp, q = e - c * rp;
      *reinterpret_cast<float4*>(L + P.dst + PER * q + c * P.ld_dst) = z;
    }
    return;
  }
  const int tr = (P.rows + 31) / 32, tc = (P.cols + 31) / 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int t = bx; t < tr * tc; t += gx) {
    const int r0 = (t % tr) * 32, c0 = (t / tr) * 32;
    if (sizeof(C) == 8 && !P.trans) {
      // complex64: lane (tp, cc) converts rows 2tp, 2tp + 1 of columns cc and
      // cc + 16 and stores each pair with one 16-byte store (blocks start at
      // even rows of even-height panels; the row after an odd last row is
      // the panel's padding row and gets zero).  Loads as below.
      const int tp = threadIdx.x & 15, cc = threadIdx.x >> 4;
      double2 v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + 2 * tp + (q & 1), c = c0 + cc + 16 * (q >> 1);
        const bool in = r < P.rows && c < P.cols;
        v[q] = K[P.src + (in ? r + (int64_t)c * P.rows : 0)];
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = r0 + 2 * tp, c = c0 + cc + 16 * h;
        if (r < P.rows && c < P.cols) {
          const bool two = r + 1 < P.rows;
          float4 o;
          o.x = (float)v[2 * h].x;
          o.y = (float)v[2 * h].y;
          o.z = two ? (float)v[2 * h + 1].x : 0.f;
          o.w = two ? (float)v[2 * h + 1].y : 0.f;
          *reinterpret_cast<float4*>(L + P.dst + r + (int64_t)c * P.ld_dst) = o;
        }
      }
    } else if (!P.trans) {
      // the four loads of a thread go out together (unconditional, from a
      // valid address outside the block), then the stores
      double2 v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + tx, c = c0 + ty + 8 * q;
        const bool in = r < P.rows && c < P.cols;
        v[q] = K[P.src + (in ? r + (int64_t)c * P.rows : 0)];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + tx, c = c0 + ty + 8 * q;
        if (r < P.rows && c < P.cols) {
          C o;
          o.x = (T)v[q].x;
          o.y = (T)v[q].y;
          L[P.dst + r + (int64_t)c * P.ld_dst] = o;
        }
      }
    } else {
      // dst(r, c) = src[c + r * cols]: read src rows c contiguous
      __syncthreads();
      double2 v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + ty + 8 * q, c = c0 + tx;
        const bool in = r < P.rows && c < P.cols;
        v[q] = K[P.src + (in ? c + (int64_t)r * P.cols : 0)];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        asm volatile("" : "+v"(v[q].x), "+v"(v[q].y));  // keeps the loads together, not sunk into the branches
        const int rr = ty + 8 * q;
        if (r0 + rr < P.rows && c0 + tx < P.cols) tileb[rr][tx] = v[q];
      }
      __syncthreads();
      if constexpr (sizeof(C) == 8) {
        // row pairs with 16-byte stores, as in the untransposed case
        const int tp = threadIdx.x & 15, c16 = threadIdx.x >> 4;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int cc = c16 + 16 * h, r = r0 + 2 * tp, c = c0 + cc;
          if (r < P.rows && c < P.cols) {
            const bool two = r + 1 < P.rows;
            const double2 v0 = tileb[2 * tp][cc], v1 = tileb[2 * tp + 1][cc];
            float4 o;
            o.x = (float)v0.x;
            o.y = (float)v0.y;
            o.z = two ? (float)v1.x : 0.f;
            o.w = two ? (float)v1.y : 0.f;
            *reinterpret_cast<float4*>(L + P.dst + r + (int64_t)c * P.ld_dst) = o;
          }
        }
      } else {
        for (int cc = ty; cc < 32; cc += 8) {
          int r = r0 + tx, c = c0 + cc;
          if (r < P.rows && c < P.cols) {
            double2 v = tileb[tx][cc];
            C o;
            o.x = (T)v.x;
            o.y = (T)v.y;
            L[P.dst + r + (int64_t)c * P.ld_dst] = o;
          }
        }
      }
    }
  }
}

// ||K||_inf: row sums of |k_ij| of the symmetric K, then the maximum.  One
// workgroup per row tile.  Every access runs along the stored blocks' unit
// stride: blocks read by columns (K_IJ, and the lower part of the diagonal
// block) with lanes over rows, blocks read by rows (K_JI^T, and the upper
// part of the diagonal block from its lower triangle) with lanes over
// columns.  Partial sums are combined in a fixed order (deterministic).
// (workgroup of 512 threads, row tile t)
__device__ __forceinline__ void knorm_part(const double2* K, const UserView& uv, const RTaskDev t, IrCtrl* ctrl) {
  const int I = t.I, nI = uv.n[I];
  __shared__ double part[5][kTileMax];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // s += |K[base + p * stride]| for p = p0, p0 + step, .. < pend, in that
  // order; eight loads go out together (from a valid address past pend)
  // and the terms past pend add zero, so the loads stay unconditional
  auto sum = [&](double& s, int64_t base, int64_t stride, int p0, int pend, int step) {
    constexpr int U = 8;
    for (int q = p0; q < pend; q += U * step) {
      double2 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int p = q + u * step;
        v[u] = K[base + (int64_t)(p < pend ? p : p0) * stride];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double a = sqrt(v[u].x * v[u].x + v[u].y * v[u].y);
        s += (q + u * step < pend) ? a : 0.0;
      }
    }
  };
  // lanes over rows: thread (row i, group g) sums the columns p = g mod 4
  {
    const int i = tid & (kTileMax - 1), g = tid >> 7;
    double s = 0;
    if (i < t.sz) {
      const int gi = t.r0 + i;
      for (int e = uv.rptr[I]; e < uv.rptr[I + 1]; ++e) {
        const RBlkDev b = uv.rblk[e];
        if (b.mode == 2) continue;
        const int pend = b.mode == 0 ? gi + 1 : uv.n[b.J];
        sum(s, b.koff + gi, nI, g, pend, 4);
      }
    }
    part[g][i] = s;
  }
  // lanes over columns: wave w sums rows w, w + 8, ... of the row-read blocks
  for (int i = w; i < t.sz; i += 8) {
    const int gi = t.r0 + i;
    double s = 0;
    for (int e = uv.rptr[I]; e < uv.rptr[I + 1]; ++e) {
      const RBlkDev b = uv.rblk[e];
      if (b.mode == 1) continue;
      if (b.mode == 2) {
        const int nJ = uv.n[b.J];
        sum(s, b.koff + (int64_t)gi * nJ, 1, lane, nJ, 64);
      } else {
        sum(s, b.koff + (int64_t)gi * nI, 1, gi + 1 + lane, nI, 64);  // (gi, p) above the diagonal = (p, gi)
      }
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) part[4][i] = s;
  }
  __syncthreads();
  __shared__ double rmax[8];
  double m = 0;
  if (tid < t.sz) m = (((part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid])) + part[4][tid]);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  if (lane == 0) rmax[w] = m;
  __syncthreads();
  if (tid == 0) {
    double r = 0;
    for (int q = 0; q < 8; ++q) r = fmax(r, rmax[q]);
    atomic_max_pos(&ctrl->knorm, r);
  }
}

}  // namespace d3m
