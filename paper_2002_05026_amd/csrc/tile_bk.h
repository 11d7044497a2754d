// Dense LDL^T of one diagonal tile (m <= 128) with Bunch-Kaufman pivoting:
// the sytrf of the dense factorization task of Sec. II, with the pivot
// search restricted to the tile so that the block pattern and the task DAG
// stay as they are.  Complex symmetric: transposes, never conjugates.
//
//   P A P^T = L D L^T,  L unit lower, D block diagonal with 1x1 and 2x2
//   blocks, P the tile's symmetric interchanges.
//
// Each step k (Bunch & Kaufman 1977, alpha = (1 + sqrt(17))/8, magnitudes
// |re| + |im| as in LAPACK's complex sytrf): with colmax the largest
// off-diagonal magnitude of column k (row imax), keep a_kk as a 1x1 pivot if
// |a_kk| >= alpha colmax, or if |a_kk| rowmax >= alpha colmax^2 (rowmax the
// largest off-diagonal magnitude of row imax); else take a_imax,imax as a
// 1x1 pivot if |a_imax,imax| >= alpha rowmax; else the 2x2 pivot of rows k
// and imax.  The interchange moves rows and columns inside the tile
// (the tile's already computed columns included); rows of the tile in
// columns left of it and the columns of the rows below it are handled by the
// callers (they keep the original order and the tile's TRSM applies P).
//
// One 512-thread workgroup, the tile in LDS (lower block triangle, the
// layout of tile_ldlt), unblocked right-looking: wave 0 chooses the pivot
// (wave-wide argmax), all threads interchange and update the trailing
// triangle.  Then L (strictly below the diagonal; a 2x2 pivot at k keeps
// D(k+1, k) in the slot of L(k+1, k), which is zero), D's diagonal, D's
// off-diagonal (doff) and the permutation (ipiv: original position of the
// unknown at each position) go out, and
//   F = L^-1 P  into linv,   G = D^-1 F  into ginv
// (column-major, leading dimension ldl), which the TRSM (LD = A F^T,
// L = A G^T), the INV tasks and the solve use in place of L^-1.
#pragma once
#include "tile_ldlt.h"

namespace d3m {

// LDS: the lower block triangle, two column vectors (the elimination's
// unscaled pivot columns, later D^-1 of the pivots), and int vectors.
template <typename T> constexpr int tile_bk_lds_bytes() {
  return (TL_NBLK * 256 + 2 * kTileMax) * (int)sizeof(cpx<T>) + 3 * kTileMax * 4 + 64;
}

template <typename T> __device__ __forceinline__ T bk_abs1(cpx<T> z) { return fabs(z.x) + fabs(z.y); }

// max with the tie to the smaller index (the first maximum, as LAPACK's
// i?amax), over a wave
template <typename T> __device__ __forceinline__ void bk_wave_argmax(T& v, int& i) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const T ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(i, off);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
}
template <typename T> __device__ __forceinline__ T bk_wave_max(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const T ov = __shfl_xor(v, off);
    v = (v < ov) ? ov : v;
  }
  return v;
}

// T: arithmetic precision; TS: storage precision.  row0: internal row of
// the tile's first unknown.  A zero (or not finite) pivot records its
// position, row0 + k, in status[0] (the smallest position wins, i.e. the
// first in elimination order); ipiv maps it to the unknown.
template <typename T, typename TS>
__device__ __noinline__ void tile_bk(typename Cplx<TS>::type* a_, int64_t lda, int m, typename Cplx<TS>::type* dout_,
                        typename Cplx<TS>::type* doff_, int32_t* ipiv, typename Cplx<TS>::type* linv_,
                        typename Cplx<TS>::type* ginv_, int64_t ldl, int row0, int32_t* status, lds_char* lds) {
  D3M_LDS cpx<T>* S = reinterpret_cast<D3M_LDS cpx<T>*>(lds);
  D3M_LDS cpx<T>* wc0 = S + TL_NBLK * 256;  // column k (unscaled), then D^-1 diagonal
  D3M_LDS cpx<T>* wc1 = wc0 + kTileMax;     // column k+1 of a 2x2 pivot, then D^-1 partner
  D3M_LDS int* perm = reinterpret_cast<D3M_LDS int*>(wc1 + kTileMax);
  D3M_LDS int* stp = perm + kTileMax;       // 1 or 2 at the first row of a pivot
  D3M_LDS int* prt = stp + kTileMax;        // other row of a 2x2 pivot, or -1
  D3M_LDS int* ctl = prt + kTileMax;        // [0] step, [1] kp, [2] skip
  D3M_GLB cpx<TS>* a = gptr_mut<TS>(a_);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nb = (m + 15) >> 4;
  const int M = nb * 16;
  constexpr int kColStep = kThreads / kTileMax;
  const int ri = tid % kTileMax, cj = tid / kTileMax;
  const T alpha = (T)((1.0 + 4.1231056256176606) / 8.0);  // (1 + sqrt(17)) / 8
  wg_sync_global();
  // lower block triangle from the tile's lower triangle; identity padding
  for (int j = cj; j < M; j += kColStep) {
    if (ri >= M || (ri >> 4) < (j >> 4)) continue;
    cpx<T> v;
    if (ri < m && j < m) {
      if (ri >= j) v = cvt_cpx<T>(a[ri + (int64_t)j * lda]);
      else { v.x = 0; v.y = 0; }
    } else {
      v.x = (ri == j) ? (T)1 : (T)0;
      v.y = 0;
    }
    S[tl_at<T>(ri, j)] = v;
  }
  if (tid < kTileMax) {
    perm[tid] = tid;
    stp[tid] = 1;
    prt[tid] = -1;
  }
  __syncthreads();
  auto at = [&](int i, int j) { return tl_at<T>(i, j); };  // i >= j
  for (int k = 0; k < m;) {
    if (w == 0) {
      const T akk = bk_abs1<T>(S[at(k, k)]);
      T cm = 0;
      int ci = k;
      for (int i = k + 1 + lane; i < m; i += 64) {
        const T v = bk_abs1<T>(S[at(i, k)]);
        if (v > cm) { cm = v; ci = i; }
      }
      bk_wave_argmax(cm, ci);
      const T colmax = cm;
      const int imax = ci;
      int kstep = 1, kp = k, skip = 0;
      const T mx = (akk < colmax) ? colmax : akk;
      if (mx == (T)0) {
        skip = 1;
      } else if (akk >= alpha * colmax) {
      } else {
        T rm = 0;
        for (int j = k + lane; j < imax; j += 64) {
          const T v = bk_abs1<T>(S[at(imax, j)]);
          rm = (rm < v) ? v : rm;
        }
        for (int i = imax + 1 + lane; i < m; i += 64) {
          const T v = bk_abs1<T>(S[at(i, imax)]);
          rm = (rm < v) ? v : rm;
        }
        const T rowmax = bk_wave_max(rm);
        if (akk >= alpha * colmax * (colmax / rowmax)) {
        } else if (bk_abs1<T>(S[at(imax, imax)]) >= alpha * rowmax) {
          kp = imax;
        } else {
          kp = imax;
          kstep = 2;
        }
      }
      if (lane == 0) {
        ctl[0] = kstep;
        ctl[1] = kp;
        ctl[2] = skip;
      }
    }
    __syncthreads();
    const int kstep = __builtin_amdgcn_readfirstlane(ctl[0]);
    const int kp = __builtin_amdgcn_readfirstlane(ctl[1]);
    int skip = __builtin_amdgcn_readfirstlane(ctl[2]);
    const int kk = k + kstep - 1;
    if (kp != kk) {
      // symmetric interchange of kk < kp inside the tile (lower storage)
      if (tid < kTileMax) {
        const int j = tid;
        if (j < kk) {
          const cpx<T> x = S[at(kk, j)], y = S[at(kp, j)];
          S[at(kk, j)] = y;
          S[at(kp, j)] = x;
        }
      } else if (tid < 2 * kTileMax) {
        const int j = tid - kTileMax;
        if (j > kk && j < kp) {
          const cpx<T> x = S[at(j, kk)], y = S[at(kp, j)];
          S[at(j, kk)] = y;
          S[at(kp, j)] = x;
        }
      } else if (tid < 3 * kTileMax) {
        const int i = tid - 2 * kTileMax;
        if (i > kp && i < m) {
          const cpx<T> x = S[at(i, kk)], y = S[at(i, kp)];
          S[at(i, kk)] = y;
          S[at(i, kp)] = x;
        }
      } else if (tid == 3 * kTileMax) {
        const cpx<T> x = S[at(kk, kk)], y = S[at(kp, kp)];
        S[at(kk, kk)] = y;
        S[at(kp, kp)] = x;
        const int t = perm[kk];
        perm[kk] = perm[kp];
        perm[kp] = t;
      }
      __syncthreads();
    }
    if (kstep == 1) {
      const cpx<T> d = S[at(k, k)];
      const bool ok = (d.x != (T)0 || d.y != (T)0) && isfinite(d.x) && isfinite(d.y);
      if (!ok) skip = 1;
      if (skip) {
        if (tid == 0) {
          atomicMin(&status[0], row0 + k);  // the position; the host maps it through ipiv
          atomicAdd(&status[1], 1);
        }
      } else {
        const cpx<T> dinv = tl_inv(d);
        if (tid < m - k - 1) {
          const int i = k + 1 + tid;
          const cpx<T> wv = S[at(i, k)];
          wc0[i] = wv;
          S[at(i, k)] = tl_mul(wv, dinv);
        }
        __syncthreads();
        {
          const int i = k + 1 + (tid & (kTileMax - 1)), g = tid >> 7;
          if (i < m) {
            const cpx<T> l = S[at(i, k)];
            for (int j = k + 1 + g; j <= i; j += kColStep) {
              cpx<T> v = S[at(i, j)];
              tl_msub(v, l, wc0[j]);
              S[at(i, j)] = v;
            }
          }
        }
      }
    } else {
      const cpx<T> da = S[at(k, k)], db = S[at(k + 1, k)], dc = S[at(k + 1, k + 1)];
      const cpx<T> det = {da.x * dc.x - da.y * dc.y - (db.x * db.x - db.y * db.y),
                          da.x * dc.y + da.y * dc.x - 2 * db.x * db.y};
      const bool ok = (det.x != (T)0 || det.y != (T)0) && isfinite(det.x) && isfinite(det.y);
      if (!ok) {
        if (tid == 0) {
          atomicMin(&status[0], row0 + k);  // the position; the host maps it through ipiv
          atomicAdd(&status[1], 1);
        }
      } else {
        const cpx<T> id = tl_inv(det);
        const cpx<T> i11 = tl_mul(dc, id), i22 = tl_mul(da, id);
        cpx<T> i12 = tl_mul(db, id);
        i12.x = -i12.x;
        i12.y = -i12.y;
        if (tid < m - k - 2) {
          const int i = k + 2 + tid;
          const cpx<T> w0 = S[at(i, k)], w1 = S[at(i, k + 1)];
          wc0[i] = w0;
          wc1[i] = w1;
          cpx<T> l0 = tl_mul(w0, i11), l1 = tl_mul(w0, i12);
          const cpx<T> t0 = tl_mul(w1, i12), t1 = tl_mul(w1, i22);
          l0.x += t0.x; l0.y += t0.y;
          l1.x += t1.x; l1.y += t1.y;
          S[at(i, k)] = l0;
          S[at(i, k + 1)] = l1;
        }
        if (tid == 0) {
          stp[k] = 2;
          prt[k] = k + 1;
          prt[k + 1] = k;
        }
        __syncthreads();
        {
          const int i = k + 2 + (tid & (kTileMax - 1)), g = tid >> 7;
          if (i < m) {
            const cpx<T> l0 = S[at(i, k)], l1 = S[at(i, k + 1)];
            for (int j = k + 2 + g; j <= i; j += kColStep) {
              cpx<T> v = S[at(i, j)];
              tl_msub(v, l0, wc0[j]);
              tl_msub(v, l1, wc1[j]);
              S[at(i, j)] = v;
            }
          }
        }
      }
    }
    __syncthreads();
    k += kstep;
  }
  // L, D, D's off-diagonal and the permutation out
  {
    D3M_GLB cpx<TS>* dout = gptr_mut<TS>(dout_);
    D3M_GLB cpx<TS>* doff = gptr_mut<TS>(doff_);
    for (int j = cj; j < m; j += kColStep)
      if (ri < m && j <= ri) {
        const cpx<T> e = S[at(ri, j)];
        a[ri + (int64_t)j * lda] = cvt_cpx<TS>(e);
        if (ri == j) dout[ri] = cvt_cpx<TS>(e);
      }
    if (tid < m) {
      cpx<T> o;
      o.x = 0;
      o.y = 0;
      if (stp[tid] == 2) o = S[at(tid + 1, tid)];
      doff[tid] = cvt_cpx<TS>(o);
      ipiv[tid] = perm[tid];
    }
  }
  __syncthreads();
  // D^-1 of the pivots into wc0 (diagonal) / wc1 (partner); L(k+1, k) of a
  // 2x2 pivot back to zero
  if (tid < m) {
    const int i = tid, q = prt[i];
    if (q < 0) {
      wc0[i] = tl_inv(S[at(i, i)]);
    } else {
      const int k0 = i < q ? i : q;
      const cpx<T> da = S[at(k0, k0)], db = S[at(k0 + 1, k0)], dc = S[at(k0 + 1, k0 + 1)];
      const cpx<T> det = {da.x * dc.x - da.y * dc.y - (db.x * db.x - db.y * db.y),
                          da.x * dc.y + da.y * dc.x - 2 * db.x * db.y};
      const cpx<T> id = tl_inv(det);
      wc0[i] = tl_mul(i == k0 ? dc : da, id);
      cpx<T> p = tl_mul(db, id);
      p.x = -p.x;
      p.y = -p.y;
      wc1[i] = p;
    }
  }
  __syncthreads();
  if (tid < m && stp[tid] == 2) {
    cpx<T> z;
    z.x = 0;
    z.y = 0;
    S[at(tid + 1, tid)] = z;
  }
  __syncthreads();
  // X_b = inverse of each diagonal 16-block of L, transposed into the
  // block's upper part (the form tl_invert_store reads): wave b, lane c
  // forms column c by forward substitution
  if (w < nb && lane < 16) {
    const int b = w, c = lane, bo = tl_blk(b, b);
    cpx<T> x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      cpx<T> t;
      t.x = 0;
      t.y = 0;
#pragma unroll
      for (int q = 0; q < i; ++q) {
        const cpx<T> l = S[bo + q * 16 + i];  // L(i, q) of the block
        const cpx<T> pr = tl_mul(l, x[q]);
        t.x += pr.x;
        t.y += pr.y;
      }
      x[i].x = (i == c) ? (T)1 : ((i < c) ? (T)0 : -t.x);
      x[i].y = (i == c) ? (T)0 : ((i < c) ? (T)0 : -t.y);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (i > c) S[bo + i * 16 + c] = x[i];
  }
  __syncthreads();
  tl_invert_store<T, TS>(S, m, gptr_mut<TS>(linv_), ldl, perm, gptr_mut<TS>(ginv_), wc0, wc1, prt);
  wg_sync_global();
}

}  // namespace d3m
