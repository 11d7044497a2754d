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
// K placements first, then the blocks to zero (fill blocks that no update
// stores into, and the padding row pairs of the others); 32x32 tiles of a K
// block (the elements of a fill block) are spread over the bx-th of gx
// workgroups (256 threads).  Transposed blocks go through LDS.  Every tile
// also leaves its |k| row and column sums in part (the input of ||K||_inf,
// so that K is read once for both): the tile goes through LDS and is added
// up there.
template <typename T>
__device__ __forceinline__ void scatter_part(const double2* K, typename Cplx<T>::type* L, const KPlaceDev* kp,
                                             int nkp, const KPlaceDev* fills, double* part, int b, int bx,
                                             int gx) {
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
  // |k| sums of the tile in tileb (destination coordinates): threads 0..127
  // add rows, 128..255 columns, four lanes per row (column) over 8 entries
  // each, combined as (s0 + s1) + (s2 + s3); a diagonal block counts its
  // lower triangle, the diagonal in the row sums only
  auto tile_sums = [&](int t, int r0, int c0) {
    const int k = (threadIdx.x & 127) >> 2, sub = threadIdx.x & 3;
    const bool col = threadIdx.x >= 128;
    double sm = 0;
#pragma unroll 4
    for (int j = 8 * sub; j < 8 * sub + 8; ++j) {
      const int rr = col ? j : k, cc = col ? k : j;
      const int r = r0 + rr, c = c0 + cc;
      bool in = r < P.rows && c < P.cols;
      if (P.diag) in = in && (col ? r > c : r >= c);
      const double2 v = tileb[rr][cc];
      sm += in ? sqrt(v.x * v.x + v.y * v.y) : 0.0;
    }
    sm += __shfl_xor(sm, 1, 64);
    sm += __shfl_xor(sm, 2, 64);
    if (sub == 0) part[P.part + (int64_t)t * 64 + (col ? 32 : 0) + k] = sm;
  };
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
      __syncthreads();  // the previous tile's sums are done with tileb
#pragma unroll
      for (int q = 0; q < 4; ++q) tileb[2 * tp + (q & 1)][cc + 16 * (q >> 1)] = v[q];
      __syncthreads();
      tile_sums(t, r0, c0);
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
      __syncthreads();  // the previous tile's sums are done with tileb
#pragma unroll
      for (int q = 0; q < 4; ++q) tileb[tx][ty + 8 * q] = v[q];
      __syncthreads();
      tile_sums(t, r0, c0);
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
      tile_sums(t, r0, c0);  // the in-range entries of tileb are the tile
    }
  }
}

// ||K||_inf: the row sums of |k_ij| of the symmetric K are the sums of the
// scatter's tile sums over each row's tiles (in the order of kn.ent, so the
// result does not depend on timing), and the norm is their maximum.  Eight
// 32-row groups per workgroup of 256 threads, starting at group 8 bx.
__device__ __forceinline__ void knorm_part(const KnormDev& kn, IrCtrl* ctrl, int bx) {
  const int g = 8 * bx + (threadIdx.x >> 5), l = threadIdx.x & 31;
  double m = 0;
  if (g < kn.ngroups) {
#pragma unroll 8
    for (int e = kn.ptr[g]; e < kn.ptr[g + 1]; ++e) m += kn.part[kn.ent[e] + l];
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  __shared__ double rmax[4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) rmax[w] = m;
  __syncthreads();
  if (threadIdx.x == 0) atomic_max_pos(&ctrl->knorm, fmax(fmax(rmax[0], rmax[1]), fmax(rmax[2], rmax[3])));
}

}  // namespace d3m
