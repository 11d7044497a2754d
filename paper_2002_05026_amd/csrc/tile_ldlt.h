// Dense LDL^T of one diagonal tile (m <= 128 rows) held in LDS, the "dense
// factorization" task of Sec. II applied to a tile: no pivoting, complex
// symmetric (transposes, never conjugates).  Blocked by 16 so that one
// 512-thread workgroup needs a few dozen barriers instead of one per pivot:
//
//   for each 16-column block k:
//     wave 0: unblocked LDL^T of the 16x16 diagonal block in registers (one
//             row per lane, pivots and multipliers broadcast across lanes)
//             and, from the same multipliers in the same instructions on
//             other lanes, the inverse X_k of its unit lower factor (one
//             column per lane), kept transposed in the block's free upper
//             triangle
//     waves:  L_ik = A_ik X_k^T D_k^-1 for the blocks below (one block per
//             wave on the matrix cores)
//     all:    A_ij -= L_ik D_k L_jk^T on the trailing blocks (one 16x16x16
//             complex product per block pair on the matrix cores): column
//             k+1 at once, the other columns on waves 1..7 while wave 0
//             factors diagonal block k+1 (look-ahead)
//
// then L (strictly below the diagonal) and D (on it) go back to the tile in
// global memory, and the full inverse Linv = L^-1 (m x m, column-major with
// leading dimension ldl, zeros above the diagonal) is formed in place of L in
// LDS by recursive doubling over 16-block super-blocks,
//   [A 0; C D]^-1 = [A^-1 0; -D^-1 C A^-1  D^-1],
// and then written out.  Rows/columns beyond m are padded with the identity.
#pragma once
#include "gemm_engine.h"

namespace d3m {

constexpr int TL_NB = kTileMax / 16;                       // 16-blocks per tile edge
constexpr int TL_NBLK = TL_NB * (TL_NB + 1) / 2;          // lower block triangle

template <typename T> constexpr int tile_ldlt_lds_bytes() {
  return (TL_NBLK * 256 + kTileMax) * (int)sizeof(cpx<T>) + 16;
}

__device__ __forceinline__ int tl_blk(int bi, int bj) { return (bi * (bi + 1) / 2 + bj) * 256; }

template <typename T>
__device__ __forceinline__ cpx<T> tl_mul(cpx<T> a, cpx<T> b) {
  cpx<T> r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

// X_b(i, k) of the inverse of diagonal block b: 1 on the diagonal, stored
// transposed in the upper triangle, zero above.
// The element is read unconditionally (from inside the block) and selected,
// so that reads of several k-steps can be issued together.
template <typename T>
__device__ __forceinline__ cpx<T> tl_x(const D3M_LDS cpx<T>* S, int b, int i, int k) {
  const cpx<T> e = S[tl_blk(b, b) + max(i, k) * 16 + min(i, k)];  // element (row k, col i) holds X(i, k), i > k
  cpx<T> v;
  v.x = (i > k) ? e.x : ((i == k) ? (T)1 : (T)0);
  v.y = (i > k) ? e.y : (T)0;
  return v;
}

// Growth test of a factorization attempt (the fallback trigger): a pivot
// with |d| < dmin * max|A|, an entry of L with |l| > lmax, or any value that
// is not finite.
struct GrowthCheck {
  bool on;
  float dmin, lmax;
};

template <typename T, typename S> __device__ __forceinline__ cpx<T> cvt_cpx(cpx<S> v) {
  cpx<T> r;
  r.x = (T)v.x;
  r.y = (T)v.y;
  return r;
}

// value of v in lane l (l uniform across the wave)
__device__ __forceinline__ float tl_bcast(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double tl_bcast(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
template <typename T> __device__ __forceinline__ cpx<T> tl_bcast(cpx<T> v, int l) {
  cpx<T> r;
  r.x = tl_bcast(v.x, l);
  r.y = tl_bcast(v.y, l);
  return r;
}

// 1/d through one reciprocal of |d|^2: the hardware reciprocal (within one
// ulp) in FP32, a correctly rounded division in FP64.
__device__ __forceinline__ float tl_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double tl_rcp(double x) { return 1.0 / x; }
template <typename T> __device__ __forceinline__ cpx<T> tl_inv(cpx<T> d) {
  const T s = tl_rcp(d.x * d.x + d.y * d.y);
  cpx<T> r;
  r.x = d.x * s;
  r.y = -d.y * s;
  return r;
}

// v -= a * b (four fused multiply-adds)
template <typename T> __device__ __forceinline__ void tl_msub(cpx<T>& v, cpx<T> a, cpx<T> b) {
  v.x = fma(-a.x, b.x, v.x);
  v.x = fma(a.y, b.y, v.x);
  v.y = fma(-a.x, b.y, v.y);
  v.y = fma(-a.y, b.x, v.y);
}

// Element (i, j), i >= j, of the lower block triangle.
template <typename T> __device__ __forceinline__ int tl_at(int i, int j) {
  return tl_blk(i >> 4, j >> 4) + (j & 15) * 16 + (i & 15);
}

// Linv = L^-1 of the unit lower tile held in S (lower block triangle; the
// inverse X_b of each diagonal 16-block kept transposed in that block's
// upper part, see tl_x), formed in place of L, then written out:
//   linv(i, col(j)) = Linv(i, j),   col(j) = perm ? perm[j] : j,
// zeros above the block diagonal.  With ginv (and D^-1 of the pivots: row
// i of D^-1 holds dinv[i] at column i and dpart[i] at column prt[i], the
// other row of a 2x2 pivot, or prt[i] = -1) also
//   ginv(i, col(j)) = sum_i' D^-1(i, i') Linv(i', j).
// Every thread of the workgroup calls.
template <typename T, typename TS>
__device__ __forceinline__ void tl_invert_store(D3M_LDS cpx<T>* S, int m, D3M_GLB cpx<TS>* linv, int64_t ldl,
                                                const D3M_LDS int* perm, D3M_GLB cpx<TS>* ginv,
                                                const D3M_LDS cpx<T>* dinv, const D3M_LDS cpx<T>* dpart,
                                                const D3M_LDS int* prt) {
  typedef typename V4<T>::type v4;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int nb = (m + 15) >> 4;
  constexpr int kColStep = kThreads / kTileMax;
  const int ri = tid % kTileMax, cj = tid / kTileMax;
  const int cjs = __builtin_amdgcn_readfirstlane(cj);
  // Linv in place of L by recursive doubling.  At level s = 1, 2, 4 (in
  // 16-blocks), pairs of already inverted diagonal super-blocks A = blocks
  // [a0, a0 + s) and D = [d0, min(d0 + s, nb)), d0 = a0 + s, turn the block
  // C = L(D, A) below them into Linv(D, A) = -D^-1 C A^-1: first P = C A^-1
  // (in place of C), then -D^-1 P.  A level has at most 16 output blocks,
  // two per wave, so the serial depth is three levels of a few block
  // products each (X_i = Linv_ii, kept transposed in the diagonal blocks).
  // Only the 4-block level has 16: wave w takes blocks w and 15 - w, i.e.
  // (i, j) and its mirror in the 4 x 4 block C, whose products
  // (a0 + 4 - j for P, i - d0 + 1 for the rest) sum to the same for every
  // wave.
  for (int sl = 1; sl < nb; sl *= 2) {
    const int npair = (nb - sl + 2 * sl - 1) / (2 * sl);  // pairs with d0 < nb
    const int tot = npair * sl * sl;
    auto blk = [&](int e, int& i, int& j, int& a0, int& d0) {
      const int q = e / (sl * sl), r = e - q * sl * sl;
      a0 = 2 * sl * q;
      d0 = a0 + sl;
      i = d0 + r / sl;
      j = a0 + r % sl;
      return e < tot && i < nb;
    };
    v4 re[2], im[2];
    // P(i, j) = sum_{j <= q < a0 + s} C(i, q) A^-1(q, j)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      re[u] = v4{0, 0, 0, 0};
      im[u] = v4{0, 0, 0, 0};
      int i, j, a0, d0;
      if (blk(u ? 15 - w : w, i, j, a0, d0))
        for (int q = j; q < a0 + sl; ++q) {
#pragma unroll
          for (int kk = 0; kk < 16; kk += 4) {
            const int kq = kk + lk;
            const cpx<T> av = S[tl_blk(i, q) + kq * 16 + lr];                              // C(i,q)(lr, kq)
            const cpx<T> bv = (q == j) ? tl_x(S, j, kq, lr) : S[tl_blk(q, j) + lr * 16 + kq];  // A^-1(q,j)(kq, lr)
            re[u] = mfma16(av.x, bv.x, re[u]);
            re[u] = mfma16(-av.y, bv.y, re[u]);
            im[u] = mfma16(av.x, bv.y, im[u]);
            im[u] = mfma16(av.y, bv.x, im[u]);
          }
        }
    }
    __syncthreads();  // every C read
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      int i, j, a0, d0;
      if (blk(u ? 15 - w : w, i, j, a0, d0))
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          cpx<T> t;
          t.x = re[u][v];
          t.y = im[u][v];
          S[tl_blk(i, j) + lr * 16 + acc_row<T>(lk, v)] = t;
        }
    }
    __syncthreads();  // P in place
    // Linv(i, j) = -sum_{d0 <= q <= i} D^-1(i, q) P(q, j)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      re[u] = v4{0, 0, 0, 0};
      im[u] = v4{0, 0, 0, 0};
      int i, j, a0, d0;
      if (blk(u ? 15 - w : w, i, j, a0, d0))
        for (int q = d0; q <= i; ++q) {
#pragma unroll
          for (int kk = 0; kk < 16; kk += 4) {
            const int kq = kk + lk;
            const cpx<T> av = (q == i) ? tl_x(S, i, lr, kq) : S[tl_blk(i, q) + kq * 16 + lr];  // D^-1(i,q)(lr, kq)
            const cpx<T> bv = S[tl_blk(q, j) + lr * 16 + kq];                                  // P(q,j)(kq, lr)
            re[u] = mfma16(av.x, bv.x, re[u]);
            re[u] = mfma16(-av.y, bv.y, re[u]);
            im[u] = mfma16(av.x, bv.y, im[u]);
            im[u] = mfma16(av.y, bv.x, im[u]);
          }
        }
    }
    __syncthreads();  // every P read
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      int i, j, a0, d0;
      if (blk(u ? 15 - w : w, i, j, a0, d0))
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          cpx<T> t;
          t.x = -re[u][v];
          t.y = -im[u][v];
          S[tl_blk(i, j) + lr * 16 + acc_row<T>(lk, v)] = t;
        }
    }
    __syncthreads();
  }
  // Linv out: zeros above the block diagonal, X_i on it, the blocks below
  // (each read at an address inside the lower block triangle, then selected)
  auto lval = [&](int i, int j, cpx<T> e) {
    const int bi = i >> 4, bj = j >> 4;
    cpx<T> v;
    const bool keep = bi > bj || (bi == bj && (i & 15) > (j & 15));
    v.x = keep ? e.x : ((i == j) ? (T)1 : (T)0);
    v.y = keep ? e.y : (T)0;
    return v;
  };
  auto laddr = [&](int i, int j) {
    const int bi = i >> 4, bj = j >> 4;
    return (bi > bj) ? tl_at<T>(i, j)
                     : (bi == bj) ? tl_blk(bi, bi) + max(i & 15, j & 15) * 16 + min(i & 15, j & 15) : tl_at<T>(i, i);
  };
  for (int j0 = cjs; j0 < m; j0 += 8 * kColStep) {
    cpx<T> e[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) e[u] = S[laddr(ri, j0 + kColStep * u)];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + kColStep * u;
      if (!(ri < m && j < m)) continue;
      const cpx<T> v = lval(ri, j, e[u]);
      const int64_t col = perm ? perm[j] : j;
      linv[ri + col * ldl] = cvt_cpx<TS>(v);
      if (ginv) {
        cpx<T> g = tl_mul(dinv[ri], v);
        const int q = prt[ri];
        if (q >= 0) {
          const cpx<T> eq = S[laddr(q, j)];
          const cpx<T> vq = lval(q, j, eq);
          const cpx<T> t = tl_mul(dpart[ri], vq);
          g.x += t.x;
          g.y += t.y;
        }
        ginv[ri + col * ldl] = cvt_cpx<TS>(g);
      }
    }
  }
}

// T: arithmetic precision; TS: storage precision of the tile, D and Linv.
// Returns true (and writes nothing back) when the growth check is on and
// trips; bad pivots are only recorded when the check is off.
template <typename T, typename TS>
__device__ bool tile_ldlt(typename Cplx<TS>::type* a_, int64_t lda, int m, typename Cplx<TS>::type* dout_,
                          typename Cplx<TS>::type* linv_, int64_t ldl, int row0, int32_t* status, float* gmin_d,
                          float* gmax_l, GrowthCheck gc, lds_char* lds) {
  typedef typename V4<T>::type v4;
  D3M_LDS cpx<T>* S = reinterpret_cast<D3M_LDS cpx<T>*>(lds);
  D3M_LDS cpx<T>* dv = S + TL_NBLK * 256;
  D3M_LDS int* flags = reinterpret_cast<D3M_LDS int*>(dv + kTileMax);  // [0] max|A| bits, [1] min|d| bits, [2] max|L| bits, [3] bad
  D3M_GLB cpx<TS>* a = gptr_mut<TS>(a_);
  D3M_GLB cpx<TS>* dout = gptr_mut<TS>(dout_);
  D3M_GLB cpx<TS>* linv = gptr_mut<TS>(linv_);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int nb = (m + 15) >> 4;
  const int M = nb * 16;
  // element loops: thread -> row ri (coalesced in global memory), columns
  // cj, cj + 4, ...
  constexpr int kColStep = kThreads / kTileMax;
  const int ri = tid % kTileMax, cj = tid / kTileMax;
  wg_sync_global();
  if (tid < 4) flags[tid] = (tid == 1) ? 0x7f800000 : 0;
  __syncthreads();
  // lower block triangle from the tile's lower triangle; identity padding.
  // Loads are issued in batches so that their latencies overlap.
  {
    constexpr int U = sizeof(cpx<TS>) == 8 ? 32 : 16;  // one batch of loads for a 128-row complex64 tile
    float amax = 0.f;  // max |A|^2 (an overflow to inf only makes the check trip)
    for (int j0 = 0; j0 < M; j0 += kColStep * U) {
      cpx<TS> buf[U];
      // unconditional loads (element 0 stands in outside the lower
      // triangle): a load under a branch gets a wait for all earlier loads
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + cj + kColStep * u;
        const bool in = ri < m && j < m && ri >= j;
        buf[u] = a[in ? ri + (int64_t)j * lda : 0];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + cj + kColStep * u;
        if (ri >= M || j >= M || (ri >> 4) < (j >> 4)) continue;
        cpx<T> v;
        if (ri < m && j < m) {
          if (ri >= j) {
            v = cvt_cpx<T>(buf[u]);
            amax = fmaxf(amax, (float)(v.x * v.x + v.y * v.y));
          } else { v.x = 0; v.y = 0; }  // upper part of a diagonal block: scratch
        } else {
          v.x = (ri == j) ? (T)1 : (T)0;
          v.y = 0;
        }
        S[tl_at<T>(ri, j)] = v;
      }
    }
    if (gc.on) atomicMax((int*)(flags), __float_as_int(sqrtf(amax)));
  }
  __syncthreads();
  // trailing update of block (gi, gj) by step k on the matrix cores:
  // A_ij -= L_ik D_k L_jk^T
  auto upd = [&](int k, int gi, int gj) {
    const int boi = tl_blk(gi, k), boj = tl_blk(gj, k);
    v4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int kq = kk + lk;
      const cpx<T> av = tl_mul(S[boi + kq * 16 + lr], dv[k * 16 + kq]);
      const cpx<T> bv = S[boj + kq * 16 + lr];
      re = mfma16(av.x, bv.x, re);
      re = mfma16(-av.y, bv.y, re);
      im = mfma16(av.x, bv.y, im);
      im = mfma16(av.y, bv.x, im);
    }
    const int bo = tl_blk(gi, gj);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = acc_row<T>(lk, v);
      cpx<T> x = S[bo + lr * 16 + r];
      x.x -= re[v];
      x.y -= im[v];
      S[bo + lr * 16 + r] = x;
    }
  };
  // Step kb: wave 0 factors diagonal block kb while waves 1..7 apply the
  // rest of step kb-1's trailing update (columns kb+1 and beyond); then the
  // blocks below, L_ik; then step kb's update of column kb+1 only, which the
  // next diagonal block and its L_ik need.  Every block still receives the
  // steps' updates in step order.
  for (int kb = 0; kb < nb; ++kb) {
    const int bkk = tl_blk(kb, kb);
    if (w == 0) {
      // Lanes 0..15 hold row r of the diagonal block, lanes 16..31 column r of
      // X (lanes 32..63 repeat them and write nothing).  Step k: pivot
      // d = A(k,k); multipliers L(c,k) = A(c,k)/d come from lane c; then for
      // c > k one instruction stream does A(r,c) -= A(r,k) L(c,k) on the row
      // lanes and X(c,r) -= X(k,r) L(c,k) on the column lanes (X(k,r) is
      // final once step k is reached).
      // (r is made opaque so that the per-lane constants below are not
      // hoisted out of the kb loop into registers held across it)
      int r = lr;
      asm volatile("" : "+v"(r));
      const bool xl = (lane & 16) != 0;
      cpx<T> v[16], dr;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const cpx<T> a = S[bkk + c * 16 + r];
        v[c].x = xl ? ((c == r) ? (T)1 : (T)0) : a.x;
        v[c].y = xl ? (T)0 : a.y;
      }
      dr.x = 1;
      dr.y = 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const cpx<T> d = tl_bcast(v[k], k);
        if (r == k) dr = d;
        const cpx<T> l = tl_mul(v[k], tl_inv(d));  // L(r,k) on the row lanes, r > k
#pragma unroll
        for (int c = k + 1; c < 16; ++c) tl_msub(v[c], v[k], tl_bcast(l, c));
        if (!xl && r > k) v[k] = l;
      }
      if (lane < 32) {
        // row r of the block: L(r,c) left of the diagonal and d_r on it from
        // the row lanes, X(c,r) to the right (the transposed X) from the
        // column lanes
#pragma unroll
        for (int c = 0; c < 16; ++c)
          if (xl ? (c > r) : (c <= r)) S[bkk + c * 16 + r] = (c == r) ? dr : v[c];
      }
      if (lane < 16) {
        dv[kb * 16 + r] = dr;
        if (kb * 16 + r < m) {
          const T ad = sqrt(dr.x * dr.x + dr.y * dr.y);
          const bool bad = !(ad > (T)0) || !isfinite(dr.x) || !isfinite(dr.y);
          if (gc.on) {
            if (bad) flags[3] = 1;
            else atomicMin((int*)(flags + 1), __float_as_int((float)ad));
          } else {
            if (bad) {
              atomicMin(&status[0], row0 + kb * 16 + r);
              atomicAdd(&status[1], 1);
            }
            if (gmin_d) atomicMin(reinterpret_cast<int*>(gmin_d), __float_as_int((float)ad));
          }
        }
      }
    } else if (kb > 0) {
      // pairs (gi, gj), gi >= gj >= kb + 1, over waves 1..7
      const int nt = nb - kb - 1;
      const int npair = nt * (nt + 1) / 2;
      for (int pr = w - 1; pr < npair; pr += kThreads / 64 - 1) {
        int bi = 0, rem = pr;
        while (rem > bi) { rem -= bi + 1; ++bi; }
        upd(kb - 1, kb + 1 + bi, kb + 1 + rem);
      }
    }
    __syncthreads();
    // L_ik = A_ik X_k^T D_k^-1 for block rows i > kb, one block per wave;
    // each wave overwrites only the block it read
    if (w < nb - kb - 1) {
      const int bo = tl_blk(kb + 1 + w, kb);
      v4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4) {
        const int kq = kk + lk;
        const cpx<T> av = S[bo + kq * 16 + lr];  // A_ik(lr, kq)
        const cpx<T> bv = tl_x(S, kb, lr, kq);   // B(kq, lr) = X_k(lr, kq)
        re = mfma16(av.x, bv.x, re);
        re = mfma16(-av.y, bv.y, re);
        im = mfma16(av.x, bv.y, im);
        im = mfma16(av.y, bv.x, im);
      }
      const cpx<T> dinv = tl_inv(dv[kb * 16 + lr]);  // column lr of the result
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        cpx<T> t;
        t.x = re[v];
        t.y = im[v];
        S[bo + lr * 16 + acc_row<T>(lk, v)] = tl_mul(t, dinv);
      }
    }
    __syncthreads();
    // step kb's update of column kb + 1: blocks (gi, kb + 1), gi >= kb + 1
    if (kb + 1 < nb) {
      for (int gi = kb + 1 + w; gi < nb; gi += kThreads / 64) upd(kb, gi, kb + 1);
      __syncthreads();
    }
  }
  // Element loops over a row's lower triangle: the 64 rows of a wave are
  // consecutive, so one past the wave's last row bounds the columns of all
  // its lanes; reads are clamped into the row and issued eight at a time.
  const int cjs = __builtin_amdgcn_readfirstlane(cj);
  const int jend = __builtin_amdgcn_readfirstlane(min(m, (ri | 63) + 1));
  if (gc.on) {
    float lm = 0.f;  // max |L|^2
    bool nf = false;
    for (int j0 = cjs; j0 < jend; j0 += 8 * kColStep) {
      cpx<T> e[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) e[u] = S[tl_at<T>(ri, min(j0 + kColStep * u, ri))];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (!(ri < m && j0 + kColStep * u < ri)) continue;
        const float sq = (float)(e[u].x * e[u].x + e[u].y * e[u].y);
        if (!(sq <= 3.0e38f)) nf = true;  // not finite (or |l| beyond 1.7e19)
        else lm = fmaxf(lm, sq);
      }
    }
    atomicMax((int*)(flags + 2), __float_as_int(sqrtf(lm)));
    if (nf) flags[3] = 1;
    __syncthreads();
    const float fa = __int_as_float(flags[0]), fd = __int_as_float(flags[1]), fl = __int_as_float(flags[2]);
    const bool trip = flags[3] != 0 || fd < gc.dmin * fa || fl > gc.lmax;
    __syncthreads();
    if (trip) return true;
    if (tid == 0 && gmin_d) atomicMin(reinterpret_cast<int*>(gmin_d), __float_as_int(fd));
  }
  // L and D back to the tile; D to dout
  {
    float lmax = 0.f;  // max |L|^2
    for (int j0 = cjs; j0 < jend; j0 += 8 * kColStep) {
      cpx<T> e[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) e[u] = S[tl_at<T>(ri, min(j0 + kColStep * u, ri))];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = j0 + kColStep * u;
        if (!(ri < m && j <= ri)) continue;
        a[ri + (int64_t)j * lda] = cvt_cpx<TS>(e[u]);
        if (ri == j) dout[ri] = cvt_cpx<TS>(e[u]);
        else lmax = fmaxf(lmax, (float)(e[u].x * e[u].x + e[u].y * e[u].y));
      }
    }
    if (gmax_l) atomicMax(reinterpret_cast<int*>(gmax_l), __float_as_int(sqrtf(lmax)));
  }
  tl_invert_store<T, TS>(S, m, linv, ldl, nullptr, nullptr, nullptr, nullptr, nullptr);
  wg_sync_global();
  return false;
}

}  // namespace d3m
