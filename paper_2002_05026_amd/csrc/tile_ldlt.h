// Dense LDL^T of one diagonal tile (m <= 128 rows) held in LDS, the "dense
// factorization" task of Sec. II applied to a tile: no pivoting, complex
// symmetric (transposes, never conjugates).  Blocked by 16 so that one
// 512-thread workgroup needs a few dozen barriers instead of one per pivot:
//
//   for each 16-column block k:
//     wave 0: unblocked LDL^T of the 16x16 diagonal block and the inverse
//             X_k of its unit lower factor (kept transposed in the block's
//             free upper triangle)
//     all:    L_ik = A_ik X_k^T D_k^-1 for the blocks below
//     all:    A_ij -= L_ik D_k L_jk^T on the trailing blocks (one 16x16x16
//             complex product per block pair on the matrix cores)
//
// then L (strictly below the diagonal) and D (on it) go back to the tile in
// global memory, and the full inverse Linv = L^-1 (m x m, column-major with
// leading dimension ldl, zeros above the diagonal) is assembled by block
// diagonals:
//   Linv_ij = -X_i sum_{j <= q < i} L_iq Linv_qj.
// Rows/columns beyond m are padded with the identity.
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
template <typename T>
__device__ __forceinline__ cpx<T> tl_x(const D3M_LDS cpx<T>* S, int b, int i, int k) {
  cpx<T> v;
  if (i == k) { v.x = 1; v.y = 0; }
  else if (i > k) v = S[tl_blk(b, b) + i * 16 + k];  // element (row k, col i) holds X(i, k)
  else { v.x = 0; v.y = 0; }
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
  const int nb = (m + 15) >> 4;
  const int M = nb * 16;
  wg_sync_global();
  if (tid < 4) flags[tid] = (tid == 1) ? 0x7f800000 : 0;
  __syncthreads();
  // lower block triangle from the tile's lower triangle; identity padding
  float amax = 0.f;
  for (int e = tid; e < M * M; e += kThreads) {
    const int i = e % M, j = e / M;
    if ((i >> 4) < (j >> 4)) continue;
    cpx<T> v;
    if (i < m && j < m) {
      if (i >= j) {
        v = cvt_cpx<T>(a[i + (int64_t)j * lda]);
        amax = fmaxf(amax, (float)sqrt(v.x * v.x + v.y * v.y));
      } else { v.x = 0; v.y = 0; }  // upper part of a diagonal block: scratch
    } else {
      v.x = (i == j) ? (T)1 : (T)0;
      v.y = 0;
    }
    S[tl_blk(i >> 4, j >> 4) + (j & 15) * 16 + (i & 15)] = v;
  }
  if (gc.on) atomicMax((int*)(flags), __float_as_int(amax));
  __syncthreads();
  for (int kb = 0; kb < nb; ++kb) {
    const int bkk = tl_blk(kb, kb);
    if (w == 0) {
      // unblocked LDL^T of the 16x16 diagonal block
      for (int k = 0; k < 16; ++k) {
        const cpx<T> d = S[bkk + k * 16 + k];
        if (lane == 0 && kb * 16 + k < m) {
          const T ad = sqrt(d.x * d.x + d.y * d.y);
          const bool bad = !(ad > (T)0) || !isfinite(d.x) || !isfinite(d.y);
          if (gc.on) {
            if (bad) flags[3] = 1;
            else atomicMin((int*)(flags + 1), __float_as_int((float)ad));
          } else {
            if (bad) {
              atomicMin(&status[0], row0 + kb * 16 + k);
              atomicAdd(&status[1], 1);
            }
            if (gmin_d) atomicMin(reinterpret_cast<int*>(gmin_d), __float_as_int((float)ad));
          }
        }
        const T den = d.x * d.x + d.y * d.y;
        cpx<T> dinv;
        dinv.x = d.x / den;
        dinv.y = -d.y / den;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int e = lane + 64 * t, r = e & 15, c = e >> 4;
          if (c > k && r >= c) {
            const cpx<T> lr = S[bkk + k * 16 + r], lc = S[bkk + k * 16 + c];
            const cpx<T> u = tl_mul(tl_mul(lr, dinv), lc);
            cpx<T> v = S[bkk + c * 16 + r];
            v.x -= u.x;
            v.y -= u.y;
            S[bkk + c * 16 + r] = v;
          }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane > k && lane < 16) S[bkk + k * 16 + lane] = tl_mul(S[bkk + k * 16 + lane], dinv);
        __builtin_amdgcn_wave_barrier();
      }
      // X = inverse of the unit lower factor, column j by lane j, stored
      // transposed above the diagonal: S(j, i) = X(i, j)
      if (lane < 16) {
        const int j = lane;
        for (int i = j + 1; i < 16; ++i) {
          cpx<T> s = S[bkk + j * 16 + i];  // L(i, j) * X(j, j)
          for (int q = j + 1; q < i; ++q) {
            const cpx<T> l = S[bkk + q * 16 + i], x = S[bkk + q * 16 + j];  // L(i,q), X(q,j)
            const cpx<T> p = tl_mul(l, x);
            s.x += p.x;
            s.y += p.y;
          }
          s.x = -s.x;
          s.y = -s.y;
          S[bkk + i * 16 + j] = s;  // X(i, j) at (row j, col i)
        }
      }
      if (lane < 16) dv[kb * 16 + lane] = S[bkk + lane * 16 + lane];
    }
    __syncthreads();
    // L_ik = A_ik X_k^T D_k^-1 for block rows i > kb
    {
      const int nbelow = nb - kb - 1;
      cpx<T> res[4];
      int cnt = 0;
      for (int e = tid; e < nbelow * 256 && cnt < 4; e += kThreads, ++cnt) {
        const int bi = kb + 1 + (e >> 8), r = e & 15, c = (e >> 4) & 15;
        const int bo = tl_blk(bi, kb);
        cpx<T> s;
        s.x = 0;
        s.y = 0;
        for (int q = 0; q <= c; ++q) {
          const cpx<T> p = tl_mul(S[bo + q * 16 + r], tl_x(S, kb, c, q));
          s.x += p.x;
          s.y += p.y;
        }
        const cpx<T> d = dv[kb * 16 + c];
        const T den = d.x * d.x + d.y * d.y;
        cpx<T> dinv;
        dinv.x = d.x / den;
        dinv.y = -d.y / den;
        res[cnt] = tl_mul(s, dinv);
      }
      __syncthreads();
      cnt = 0;
      for (int e = tid; e < nbelow * 256 && cnt < 4; e += kThreads, ++cnt) {
        const int bi = kb + 1 + (e >> 8), r = e & 15, c = (e >> 4) & 15;
        S[tl_blk(bi, kb) + c * 16 + r] = res[cnt];
      }
    }
    __syncthreads();
    // trailing update on the matrix cores: A_ij -= L_ik D_k L_jk^T
    {
      const int nt = nb - kb - 1;
      const int npair = nt * (nt + 1) / 2;
      const int lr = lane & 15, lk = lane >> 4;
      for (int pr = w; pr < npair; pr += kThreads / 64) {
        int bi = 0, rem = pr;
        while (rem > bi) { rem -= bi + 1; ++bi; }
        const int bj = rem;  // pair (bi, bj), bi >= bj, offsets from kb+1
        const int gi = kb + 1 + bi, gj = kb + 1 + bj;
        const int boi = tl_blk(gi, kb), boj = tl_blk(gj, kb);
        v4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
          const int kq = kk + lk;
          const cpx<T> av = tl_mul(S[boi + kq * 16 + lr], dv[kb * 16 + kq]);
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
      }
    }
    __syncthreads();
  }
  if (gc.on) {
    float lm = 0.f;
    bool nf = false;
    for (int e = tid; e < m * m; e += kThreads) {
      const int i = e % m, j = e / m;
      if (i <= j) continue;
      const cpx<T> v = S[tl_blk(i >> 4, j >> 4) + (j & 15) * 16 + (i & 15)];
      const float av = (float)sqrt(v.x * v.x + v.y * v.y);
      if (!(av <= 3.0e38f)) nf = true;
      else lm = fmaxf(lm, av);
    }
    atomicMax((int*)(flags + 2), __float_as_int(lm));
    if (nf) flags[3] = 1;
    __syncthreads();
    const float fa = __int_as_float(flags[0]), fd = __int_as_float(flags[1]), fl = __int_as_float(flags[2]);
    const bool trip = flags[3] != 0 || fd < gc.dmin * fa || fl > gc.lmax;
    __syncthreads();
    if (trip) return true;
    if (tid == 0 && gmin_d) atomicMin(reinterpret_cast<int*>(gmin_d), __float_as_int(fd));
  }
  // L and D back to the tile; D to dout
  float lmax = 0.f;
  for (int e = tid; e < m * m; e += kThreads) {
    const int i = e % m, j = e / m;
    if (i < j) continue;
    const cpx<T> v = S[tl_blk(i >> 4, j >> 4) + (j & 15) * 16 + (i & 15)];
    a[i + (int64_t)j * lda] = cvt_cpx<TS>(v);
    if (i == j) dout[i] = cvt_cpx<TS>(v);
    else lmax = fmaxf(lmax, (float)sqrt(v.x * v.x + v.y * v.y));
  }
  if (gmax_l) atomicMax(reinterpret_cast<int*>(gmax_l), __float_as_int(lmax));
  // Linv: diagonal blocks and zeros above them
  for (int e = tid; e < m * m; e += kThreads) {
    const int i = e % m, j = e / m;
    if ((i >> 4) > (j >> 4)) continue;
    cpx<T> v;
    if ((i >> 4) == (j >> 4)) v = tl_x(S, i >> 4, i & 15, j & 15);
    else { v.x = 0; v.y = 0; }
    linv[i + (int64_t)j * ldl] = cvt_cpx<TS>(v);
  }
  // block diagonals d = 1.. of Linv: T = sum_q L_iq Linv_qj, Linv_ij = -X_i T
  const int lr = lane & 15, lk = lane >> 4;
  for (int dist = 1; dist < nb; ++dist) {
    wg_sync_global();
    for (int bj = w; bj + dist < nb; bj += kThreads / 64) {
      const int bi = bj + dist;
      v4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
      for (int q = bj; q < bi; ++q) {
        const int boq = tl_blk(bi, q);
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
          const int kq = kk + lk;
          const cpx<T> av = S[boq + kq * 16 + lr];  // L(bi,q)(lr, kq)
          cpx<T> bv;                               // Linv(q,bj)(kq, lr)
          if (q == bj) bv = tl_x(S, bj, kq, lr);
          else {
            const int gr = 16 * q + kq, gcl = 16 * bj + lr;
            if (gr < m && gcl < m) bv = cvt_cpx<T>(linv[gr + (int64_t)gcl * ldl]);
            else { bv.x = (gr == gcl) ? (T)1 : (T)0; bv.y = 0; }
          }
          re = mfma16(av.x, bv.x, re);
          re = mfma16(-av.y, bv.y, re);
          im = mfma16(av.x, bv.y, im);
          im = mfma16(av.y, bv.x, im);
        }
      }
      // T goes through the output block of Linv to change register layout
      const int gcl = 16 * bj + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gr = 16 * bi + acc_row<T>(lk, v);
        if (gr < m && gcl < m) {
          cpx<T> t;
          t.x = re[v];
          t.y = im[v];
          linv[gr + (int64_t)gcl * ldl] = cvt_cpx<TS>(t);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
      v4 re2 = {0, 0, 0, 0}, im2 = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4) {
        const int kq = kk + lk;
        const cpx<T> av = tl_x(S, bi, lr, kq);  // X_i(lr, kq)
        cpx<T> bv;                             // T(kq, lr)
        const int gr = 16 * bi + kq;
        if (gr < m && gcl < m) bv = cvt_cpx<T>(linv[gr + (int64_t)gcl * ldl]);
        else { bv.x = 0; bv.y = 0; }
        re2 = mfma16(av.x, bv.x, re2);
        re2 = mfma16(-av.y, bv.y, re2);
        im2 = mfma16(av.x, bv.y, im2);
        im2 = mfma16(av.y, bv.x, im2);
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gr = 16 * bi + acc_row<T>(lk, v);
        if (gr < m && gcl < m) {
          cpx<T> t;
          t.x = -re2[v];
          t.y = -im2[v];
          linv[gr + (int64_t)gcl * ldl] = cvt_cpx<TS>(t);
        }
      }
    }
  }
  wg_sync_global();
  return false;
}

}  // namespace d3m
